// ml.hip -- descriptor-MLP force surrogate on gfx950.
//
// The paper's integrator (eq. 4, eq. 8) needs a potential V; this surrogate
// supplies V = sum_i E_i with E_i a small network of per-atom descriptors:
//   f_c(r) = (cos(pi r / r_c) + 1) / 2 for r < r_c
//   radial    phi_c(r) = exp(-eta_r (r - mu_c)^2) f_c(r), 32 channels on
//             [r_min, r_c], eta_r = 1 / (2 dr^2)
//   angular   psi_k(r) = exp(-eta_a (r - nu_k)^2) f_c(r), 8 channels,
//             A1 = sum_j psi_k rhat_j, A2 = sum_j psi_k (rhat_j rhat_j^T - I/3)
//   G[b] = (sum_j phi_c, |A1|^2, ||A2||_F^2) over neighbours j of species b
//   E_i = w3 . silu(W2 silu(W1 x + b1) + b2) + b3 + e0, x = (G - mu) inv_sd
// Forces F = -dE/dr by the chain rule per pair: dE_i/dd_ij is stored for
// every neighbour-list entry, and F_k = sum_j (dE_k/dd_kj - dE_j/dd_jk)
// gathers the reverse entries in a fixed order (deterministic, no atomics).
// Training (loss on energies and forces) differentiates the forces with
// respect to the weights: a Jacobian-vector product of the descriptors with
// dL/dF, then forward mode through the network's input gradient and reverse
// mode back to the weights.
//
// Layout: one wavefront per centre (atom, bead) for the neighbour loops,
// with the pair geometry staged in LDS and the 64 lanes split over channels
// (radial: 2 pair slots x 32 channels; angular: 8 pair slots x 8 channels);
// one lane per hidden unit for the network, weights in LDS.
#include "force_epilogue.h"
#include "qtb_internal.h"

namespace qtb {
namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kPiF = 3.14159265358979323846f;

__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }

__device__ __forceinline__ float bf16f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }

// Wavefront-local LDS ordering (the lanes of one wavefront exchange data).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T> struct V4T;
template <> struct V4T<float> { using type = float4; };
template <> struct V4T<double> { using type = double4; };

template <typename T>
__device__ __forceinline__ int ebits(const typename V4T<T>::type& v);
template <>
__device__ __forceinline__ int ebits<float>(const float4& v) { return (int)__float_as_uint(v.w); }
template <>
__device__ __forceinline__ int ebits<double>(const double4& v)
{
    return (int)(uint32_t)__double_as_longlong(v.w);
}

__device__ __forceinline__ float wsum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ------------------------------------------------------- neighbour lists
// Keep the plain list's entries within r_ml + skin + dev_i + dev_j (the plain
// list holds every pair within r_cut + skin + the same margins, r_ml <= r_cut).
template <typename T>
__global__ void __launch_bounds__(256) k_ml_list(const RepDev* __restrict__ reps,
                                                 const BlockEntry* __restrict__ blocks,
                                                 int n_entries, int32_t* __restrict__ status,
                                                 const StepRef sync)
{
    using T4 = typename V4T<T>::type;
    const StepIdx si = step_index(sync);
    if (status[kAnyRebuild + si.f] == 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int e = blockIdx.x; e < n_entries; e += gridDim.x) {
        const BlockEntry be = blocks[e];
        const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
        if (R.rflag[si.f] == 0 || R.ml_nb == nullptr) continue;
        const int i = be.atom0 + wave;
        if (i >= R.N) continue;
        const double* __restrict__ devb = R.devbb[si.p];
        const T4* __restrict__ ent = (const T4*)R.nb_entries + (size_t)i * R.maxnb;
        T4* __restrict__ out = (T4*)R.ml_nb + (size_t)i * R.maxml;
        // the pair list's core entries, then its shell entries, each in scan order
        const int cnt = R.nb_count[i], ncore = R.nb_core[i];
        const double base = R.ml_rcs + devb[i];  // r_ml + skin + dev_i
        int n = 0;
        for (int k0 = 0; k0 < cnt; k0 += 64) {
            const int k = k0 + lane;
            bool hit = false;
            T4 E;
            if (k < cnt) {
                E = ent[k < ncore ? k : R.maxnb - 1 - (k - ncore)];
                const double Rij = base + devb[ebits<T>(E)];
                const double r2 = (double)E.x * E.x + (double)E.y * E.y + (double)E.z * E.z;
                hit = r2 < Rij * Rij;
            }
            const uint64_t mask = __ballot(hit);
            if (hit) {
                const int slot = n + __popcll(mask & below);
                if (slot < R.maxml) out[slot] = E;
            }
            n += __popcll(mask);
        }
        if (lane == 0) {
            R.ml_nc[i] = min(n, R.maxml);
            if (n > R.maxml) atomicOr(status, kStatusMlList);
        }
    }
}

// Slot of entry (i -> j, D) in j's list: (j -> i, -D).  Both come from the
// same FP64 displacement with its sign flipped, so the match is exact.  The
// plain list (and so this filtered one) holds its entries in ascending
// 64-atom chunks of the neighbour index, so a binary search finds i's chunk in
// j's list and a short scan of that chunk the entry; a full scan backs it up.
// One wavefront per atom over the whole block table: this runs only after a
// rebuild, and its dependent loads need the occupancy.
template <typename T>
__global__ void __launch_bounds__(256) k_ml_rev(const RepDev* __restrict__ reps,
                                                const BlockEntry* __restrict__ blocks,
                                                int n_entries, int32_t* __restrict__ status,
                                                const StepRef sync)
{
    using T4 = typename V4T<T>::type;
    const StepIdx si = step_index(sync);
    if (status[kAnyRebuild + si.f] == 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int e = blockIdx.x; e < n_entries; e += gridDim.x) {
        const BlockEntry be = blocks[e];
        const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
        if (R.rflag[si.f] == 0 || R.ml_nb == nullptr) continue;
        const int i = be.atom0 + wave;
        if (i >= R.N) continue;
        const T4* __restrict__ ent = (const T4*)R.ml_nb;
        const int cnt = R.ml_nc[i];
        const int key = i >> 6;
        for (int k = lane; k < cnt; k += 64) {
            const T4 E = ent[(size_t)i * R.maxml + k];
            const int j = ebits<T>(E);
            const int cj = R.ml_nc[j];
            const T4* __restrict__ lj = ent + (size_t)j * R.maxml;
            int lo = 0, hi = cj;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((ebits<T>(lj[mid]) >> 6) < key)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            int found = -1;
            for (int q = lo; q < cj; ++q) {
                const T4 F = lj[q];
                const int m = ebits<T>(F);
                if ((m >> 6) != key) break;
                if (m == i && F.x == -E.x && F.y == -E.y && F.z == -E.z) {
                    found = q;
                    break;
                }
            }
            for (int q = 0; found < 0 && q < cj; ++q) {
                const T4 F = lj[q];
                if (ebits<T>(F) == i && F.x == -E.x && F.y == -E.y && F.z == -E.z) found = q;
            }
            R.ml_rev[(size_t)i * R.maxml + k] = found < 0 ? 0 : found;
            if (found < 0) atomicOr(status, kStatusMlList);
        }
    }
}

// ------------------------------------------------------------ descriptors
// Stage of one chunk of up to 64 pairs within r_ml, per wavefront.
struct PairStage {
    float r[64], fc[64], dfc[64], rx[64], ry[64], rz[64], sp[64];
    float wx[64], wy[64], wz[64];  // JVP direction u_j - u_i (training)
    int slot[64];                  // list entry of the staged pair
};

// Stage the pairs of entries k0 .. k0+63 of centre (i, s); returns how many.
template <typename T, bool DIR>
__device__ __forceinline__ int stage_pairs(const RepDev& R, const MlDev& m, int i, int s,
                                           const typename V4T<T>::type ui, int k0, int cnt,
                                           PairStage& st, int lane, float wix, float wiy,
                                           float wiz, const typename V4T<T>::type* u)
{
    using T4 = typename V4T<T>::type;
    const T4* __restrict__ ent = (const T4*)R.ml_nb + (size_t)i * R.maxml;
    const int P = R.P;
    const int k = k0 + lane;
    bool hit = false;
    float dx = 0.f, dy = 0.f, dz = 0.f, r2 = 0.f;
    int j = 0;
    if (k < cnt) {
        const T4 E = ent[k];
        j = ebits<T>(E);
        const T4 Uj = u[(size_t)j * P + s];
        // entries hold c_i - c_j (+ image): d_ij = r_j - r_i = (U_j - u_i) - D
        dx = (float)((Uj.x - ui.x) - E.x);
        dy = (float)((Uj.y - ui.y) - E.y);
        dz = (float)((Uj.z - ui.z) - E.z);
        r2 = dx * dx + dy * dy + dz * dz;
        hit = r2 < m.r_cut * m.r_cut;
    }
    const uint64_t mask = __ballot(hit);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (hit) {
        const int t = __popcll(mask & below);
        const float r = __builtin_sqrtf(r2);
        const float ir = 1.0f / r;
        const float ang = kPiF * r / m.r_cut;
        st.r[t] = r;
        st.fc[t] = 0.5f * (__cosf(ang) + 1.0f);
        st.dfc[t] = -0.5f * kPiF / m.r_cut * __sinf(ang);
        st.rx[t] = dx * ir;
        st.ry[t] = dy * ir;
        st.rz[t] = dz * ir;
        st.sp[t] = (float)R.species[j];
        st.slot[t] = k;
        if (DIR) {
            const size_t N = R.N;
            const float* __restrict__ uu = R.ml_u + (size_t)s * 3 * N;
            st.wx[t] = uu[j] - wix;
            st.wy[t] = uu[N + j] - wiy;
            st.wz[t] = uu[2 * N + j] - wiz;
        }
    }
    wave_sync();
    return __popcll(mask);
}

// Centre blocks: 4 atoms (one per wavefront), one bead (BlockEntry.group).
template <typename T>
__global__ void __launch_bounds__(256) k_ml_desc(const RepDev* __restrict__ reps, const MlDev m,
                                                 const BlockEntry* __restrict__ blocks, int n_rep,
                                                 int32_t* __restrict__ status,
                                                 const StepRef sync)
{
    using T4 = typename V4T<T>::type;
    __shared__ PairStage stage[4];
    const StepIdx si = step_index(sync);
    if (blockIdx.x == 0) {  // this step's rebuild (if any) is done
        for (int r = threadIdx.x; r < n_rep; r += blockDim.x) reps[r].rflag[si.f] = 0;
        if (threadIdx.x == 0) status[kAnyRebuild + si.f] = 0;
    }
    const int lb = xcd_block();
    const BlockEntry be = blocks[lb];
    const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = be.atom0 + wave, s = be.group;
    if (i >= R.N) return;  // uniform per wavefront; no block barrier below
    PairStage& st = stage[wave];
    const int N = R.N, P = R.P;
    const T4* __restrict__ u = (const T4*)R.ub[si.p];
    const T4 ui = u[(size_t)i * P + s];
    const int cnt = R.ml_nc[i];
    // radial lanes: channel c, pair parity h; angular lanes: channel k, slot q
    const int c = lane & 31, h = lane >> 5;
    const int ka = lane & 7, qa = lane >> 3;
    const float mu_c = m.mu0 + m.dr * c;
    const float nu_k = m.nu0 + m.da * ka;
    float g0 = 0.f, g1 = 0.f;
    float a1[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    float a2[2][6] = {{0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}};
    for (int k0 = 0; k0 < cnt; k0 += 64) {
        const int n = stage_pairs<T, false>(R, m, i, s, ui, k0, cnt, st, lane, 0.f, 0.f, 0.f, u);
        for (int t = h; t < n; t += 2) {
            const float x = st.r[t] - mu_c;
            const float ph = fexp(-m.eta_r * x * x) * st.fc[t];
            const bool b1 = st.sp[t] != 0.0f;
            g0 += b1 ? 0.0f : ph;
            g1 += b1 ? ph : 0.0f;
        }
        for (int t = qa; t < n; t += 8) {
            const float x = st.r[t] - nu_k;
            const float ps = fexp(-m.eta_a * x * x) * st.fc[t];
            const float w1 = st.sp[t] != 0.0f ? ps : 0.0f;
            const float w0 = ps - w1;
            const float rx = st.rx[t], ry = st.ry[t], rz = st.rz[t];
            const float q[6] = {rx * rx - (1.0f / 3.0f), ry * ry - (1.0f / 3.0f),
                                rz * rz - (1.0f / 3.0f), rx * ry, rx * rz, ry * rz};
            a1[0][0] += w0 * rx; a1[0][1] += w0 * ry; a1[0][2] += w0 * rz;
            a1[1][0] += w1 * rx; a1[1][1] += w1 * ry; a1[1][2] += w1 * rz;
#pragma unroll
            for (int z = 0; z < 6; ++z) {
                a2[0][z] += w0 * q[z];
                a2[1][z] += w1 * q[z];
            }
        }
        wave_sync();  // the next chunk overwrites the stage
    }
    g0 += __shfl_xor(g0, 32);
    g1 += __shfl_xor(g1, 32);
#pragma unroll
    for (int off = 8; off < 64; off <<= 1) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int z = 0; z < 3; ++z) a1[b][z] += __shfl_xor(a1[b][z], off);
#pragma unroll
            for (int z = 0; z < 6; ++z) a2[b][z] += __shfl_xor(a2[b][z], off);
        }
    }
    const size_t cidx = (size_t)s * N + i;
    float* __restrict__ G = R.ml_G + cidx * kMlFeat;
    if (lane < 32) {
        G[lane] = g0;
        G[kMlFeatSp + lane] = g1;
    }
    if (lane < 8) {
        float* __restrict__ aux = R.ml_aux + cidx * kMlAux;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const float l1 = a1[b][0] * a1[b][0] + a1[b][1] * a1[b][1] + a1[b][2] * a1[b][2];
            const float l2 = a2[b][0] * a2[b][0] + a2[b][1] * a2[b][1] + a2[b][2] * a2[b][2] +
                             2.0f * (a2[b][3] * a2[b][3] + a2[b][4] * a2[b][4] + a2[b][5] * a2[b][5]);
            G[b * kMlFeatSp + kMlRad + lane] = l1;
            G[b * kMlFeatSp + kMlRad + kMlAng + lane] = l2;
            float* o = aux + (b * kMlAng + lane) * 9;
            o[0] = a1[b][0]; o[1] = a1[b][1]; o[2] = a1[b][2];
#pragma unroll
            for (int z = 0; z < 6; ++z) o[3 + z] = a2[b][z];
        }
    }
}

// ---------------------------------------------------------------- network
// Weights of both species in LDS, padded rows (97, 65) so that both the
// row-wise (forward) and column-wise (backward) reads are conflict-free.
constexpr int kW1S = kMlFeat + 1;    // 97
constexpr int kW2S = kMlHidden + 1;  // 65
constexpr int kMlpWaves = 16;

struct alignas(16) MlpLds {
    float W1[2][kMlHidden][kW1S];
    float W2[2][kMlHidden][kW2S];
    float b1[2][kMlHidden], b2[2][kMlHidden], w3[2][kMlHidden];
    float b3[4];
    float mu[2][kMlFeat], isd[2][kMlFeat];
};
static_assert(sizeof(MlpLds) % 16 == 0, "stage arrays after the weights must stay 16-byte aligned");

__device__ void load_weights(MlpLds& L, const MlDev& m)
{
    for (int t = threadIdx.x; t < 2 * kMlHidden * kMlFeat; t += blockDim.x) {
        const int a = t / (kMlHidden * kMlFeat), r = t % (kMlHidden * kMlFeat);
        L.W1[a][r / kMlFeat][r % kMlFeat] = bf16f(m.wq[a * kMlParamsSp + kMlOffW1 + r]);
    }
    for (int t = threadIdx.x; t < 2 * kMlHidden * kMlHidden; t += blockDim.x) {
        const int a = t / (kMlHidden * kMlHidden), r = t % (kMlHidden * kMlHidden);
        L.W2[a][r / kMlHidden][r % kMlHidden] = bf16f(m.wq[a * kMlParamsSp + kMlOffW2 + r]);
    }
    for (int t = threadIdx.x; t < 2 * kMlHidden; t += blockDim.x) {
        const int a = t / kMlHidden, o = t % kMlHidden;
        L.b1[a][o] = m.master[a * kMlParamsSp + kMlOffB1 + o];
        L.b2[a][o] = m.master[a * kMlParamsSp + kMlOffB2 + o];
        L.w3[a][o] = bf16f(m.wq[a * kMlParamsSp + kMlOffW3 + o]);
    }
    if (threadIdx.x < 2) L.b3[threadIdx.x] = m.master[threadIdx.x * kMlParamsSp + kMlOffB3];
    for (int t = threadIdx.x; t < 2 * kMlFeat; t += blockDim.x) {
        L.mu[t / kMlFeat][t % kMlFeat] = m.mu[t];
        L.isd[t / kMlFeat][t % kMlFeat] = m.inv_sd[t];
    }
    __syncthreads();
}

// ------------------------------------------------------ network, matrix cores
// The same network for 32 centres per wavefront on v_mfma_f32_32x32x16_bf16.
// The weights are BF16 numbers; each FP32 activation enters as three BF16
// parts hi + mid + lo (equal to it to FP32 rounding), so every product with a
// weight is exact and the sums are FP32, as in the vector form.  Both
// species' weights are applied and each centre (row) keeps its own species'
// result.  Per layer, the activations of the 32 centres sit in the
// wavefront's LDS tile T[centre][unit] (A operand rows) and the weights in
// LDS in both orientations (B operand columns).
// Operand layout of 32x32x16: lane l gives A row (l & 31) and B column
// (l & 31) for k = 8 (l >> 5) .. +7; the accumulator element r of lane l is
// C[8 (r >> 2) + 4 (l >> 5) + (r & 3)][l & 31].
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kTS = 100;    // row stride (floats) of a wavefront's activation tile
constexpr int kWR1 = 104;   // row stride (BF16) of W1 [o][f]
constexpr int kWR = 72;     // row stride (BF16) of W1T [f][o], W2 [o][k], W2T [k][o]
constexpr int kMfmaWaves = 4;

struct alignas(16) MfmaLds {
    uint16_t W1[2][kMlHidden][kWR1];
    uint16_t W1T[2][kMlFeat][kWR];
    uint16_t W2[2][kMlHidden][kWR];
    uint16_t W2T[2][kMlHidden][kWR];
    float b1[2][kMlHidden], b2[2][kMlHidden], w3[2][kMlHidden];
    float b3[4];
    float mu[2][kMlFeat], isd[2][kMlFeat];
    int sp[kMfmaWaves][32];
};
static_assert(sizeof(MfmaLds) % 16 == 0, "the activation tiles after the weights stay aligned");

__device__ __forceinline__ float bf16v(uint32_t h) { return __uint_as_float(h << 16); }

// x (8 FP32 values) as three BF16 operands with x = hi + mid + lo to FP32
// rounding (each part rounded to nearest even from the remainder).
__device__ __forceinline__ void split3(const float4 x0, const float4 x1, bf16x8& hi, bf16x8& mid,
                                       bf16x8& lo)
{
    const float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const __bf16 h = (__bf16)x[q];
        const float r = x[q] - (float)h;
        const __bf16 m = (__bf16)r;
        hi[q] = h;
        mid[q] = m;
        lo[q] = (__bf16)(r - (float)m);
    }
}

__device__ __forceinline__ bf16x8 ldb(const uint16_t* p)
{
    return __builtin_bit_cast(bf16x8, *(const u32x4*)p);
}

// acc += A . B with A the three-part activations and B one weight fragment.
__device__ __forceinline__ void mfma3(f32x16& acc, const bf16x8& hi, const bf16x8& mid,
                                      const bf16x8& lo, const bf16x8& b)
{
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi, b, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(mid, b, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo, b, acc, 0, 0, 0);
}

__device__ void load_weights_mfma(MfmaLds& L, const MlDev& m)
{
    for (int t = threadIdx.x; t < 2 * kMlHidden * kMlFeat; t += blockDim.x) {
        const int a = t / (kMlHidden * kMlFeat), r = t % (kMlHidden * kMlFeat);
        const int o = r / kMlFeat, f = r % kMlFeat;
        const uint16_t w = m.wq[a * kMlParamsSp + kMlOffW1 + r];
        L.W1[a][o][f] = w;
        L.W1T[a][f][o] = w;
    }
    for (int t = threadIdx.x; t < 2 * kMlHidden * kMlHidden; t += blockDim.x) {
        const int a = t / (kMlHidden * kMlHidden), r = t % (kMlHidden * kMlHidden);
        const int o = r / kMlHidden, k = r % kMlHidden;
        const uint16_t w = m.wq[a * kMlParamsSp + kMlOffW2 + r];
        L.W2[a][o][k] = w;
        L.W2T[a][k][o] = w;
    }
    for (int t = threadIdx.x; t < 2 * kMlHidden; t += blockDim.x) {
        const int a = t / kMlHidden, o = t % kMlHidden;
        L.b1[a][o] = m.master[a * kMlParamsSp + kMlOffB1 + o];
        L.b2[a][o] = m.master[a * kMlParamsSp + kMlOffB2 + o];
        L.w3[a][o] = bf16f(m.wq[a * kMlParamsSp + kMlOffW3 + o]);
    }
    if (threadIdx.x < 2) L.b3[threadIdx.x] = m.master[threadIdx.x * kMlParamsSp + kMlOffB3];
    for (int t = threadIdx.x; t < 2 * kMlFeat; t += blockDim.x) {
        L.mu[t / kMlFeat][t % kMlFeat] = m.mu[t];
        L.isd[t / kMlFeat][t % kMlFeat] = m.inv_sd[t];
    }
    __syncthreads();
}

// Network blocks: BlockEntry {rep, first centre (s N + i), count <= 64}; each
// holds two tiles of 32 centres, one wavefront per tile.  Outputs the atomic
// energy (without e0) and dE/dG.
__global__ void __launch_bounds__(256) k_ml_mlp_mfma(const RepDev* __restrict__ reps,
                                                     const MlDev m,
                                                     const BlockEntry* __restrict__ blocks,
                                                     int n_blocks)
{
    extern __shared__ float4 lds_raw[];
    MfmaLds& L = *reinterpret_cast<MfmaLds*>(lds_raw);
    load_weights_mfma(L, m);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 31, lk = lane >> 5;
    float (*T)[kTS] = reinterpret_cast<float (*)[kTS]>(reinterpret_cast<char*>(lds_raw) +
                                                     sizeof(MfmaLds) +
                                                     sizeof(float) * 32 * kTS * wave);
    int* spw = L.sp[wave];
    const int n_tiles = 2 * n_blocks;
    for (int t = blockIdx.x * kMfmaWaves + wave; t < n_tiles; t += gridDim.x * kMfmaWaves) {
        const BlockEntry be = blocks[t >> 1];
        const int c0 = 32 * (t & 1);
        if (c0 >= be.group) continue;  // uniform per wavefront
        const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
        const int N = R.N;
        const int nv = min(32, be.group - c0);
        const int cbase = be.atom0 + c0;  // centre of row q: cbase + (q < nv ? q : 0)
        if (lane < 32) spw[lane] = R.species[(cbase + (lane < nv ? lane : 0)) % N];
        wave_sync();
        {
            // all 48 loads of a lane in flight at once (one wavefront per SIMD)
            float gv[32][2];
#pragma unroll
            for (int q = 0; q < 32; ++q) {
                const float* __restrict__ g = R.ml_G + (size_t)(cbase + (q < nv ? q : 0)) * kMlFeat;
                gv[q][0] = g[lane];
                gv[q][1] = lane < kMlFeat - 64 ? g[64 + lane] : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < 32; ++q) {
                const int a = spw[q];
                T[q][lane] = (gv[q][0] - L.mu[a][lane]) * L.isd[a][lane];
                if (lane < kMlFeat - 64)
                    T[q][64 + lane] = (gv[q][1] - L.mu[a][64 + lane]) * L.isd[a][64 + lane];
            }
        }
        // species of the accumulator rows of this lane: bit r set for species 1
        uint32_t s1m = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r)
            s1m |= (uint32_t)(spw[8 * (r >> 2) + 4 * lk + (r & 3)] != 0) << r;
        wave_sync();
        f32x16 acc[2][2];
        bf16x8 ah, am, al;
        // layer 1: z1[c][o] = sum_f x[c][f] W1[o][f]
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][nt][r] = 0.0f;
#pragma unroll
        for (int ks = 0; ks < kMlFeat / 16; ++ks) {
            const int k0 = 16 * ks + 8 * lk;
            split3(*(const float4*)&T[li][k0], *(const float4*)&T[li][k0 + 4], ah, am, al);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    mfma3(acc[a][nt], ah, am, al, ldb(&L.W1[a][32 * nt + li][k0]));
        }
        wave_sync();  // all rows read before the tile is overwritten
        float s1v[2][16];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int q = 8 * (r >> 2) + 4 * lk + (r & 3), o = 32 * nt + li;
                const int a = (s1m >> r) & 1;
                const float z = (a ? acc[1][nt][r] : acc[0][nt][r]) + L.b1[a][o];
                const float sg = sigm(z);
                s1v[nt][r] = sg * (1.0f + z * (1.0f - sg));
                T[q][o] = z * sg;
            }
        wave_sync();
        // layer 2: z2[c][o] = sum_k h1[c][k] W2[o][k]
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][nt][r] = 0.0f;
#pragma unroll
        for (int ks = 0; ks < kMlHidden / 16; ++ks) {
            const int k0 = 16 * ks + 8 * lk;
            split3(*(const float4*)&T[li][k0], *(const float4*)&T[li][k0 + 4], ah, am, al);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    mfma3(acc[a][nt], ah, am, al, ldb(&L.W2[a][32 * nt + li][k0]));
        }
        wave_sync();
        float d2v[2][16];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int q = 8 * (r >> 2) + 4 * lk + (r & 3), o = 32 * nt + li;
                const int a = (s1m >> r) & 1;
                const float z = (a ? acc[1][nt][r] : acc[0][nt][r]) + L.b2[a][o];
                const float sg = sigm(z);
                const float w3 = L.w3[a][o];
                d2v[nt][r] = w3 * sg * (1.0f + z * (1.0f - sg));
                T[q][o] = w3 * (z * sg);
            }
        wave_sync();
        if (lane < nv) {  // E_i - b3 - e0 = sum_o w3 h2, in unit order
            float y = 0.0f;
            for (int o = 0; o < kMlHidden; ++o) y += T[lane][o];
            R.ml_y[cbase + lane] = y + L.b3[spw[lane]];
        }
        wave_sync();
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int r = 0; r < 16; ++r) T[8 * (r >> 2) + 4 * lk + (r & 3)][32 * nt + li] = d2v[nt][r];
        wave_sync();
        // delta1[c][k] = s1[c][k] sum_o delta2[c][o] W2[o][k]
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][nt][r] = 0.0f;
#pragma unroll
        for (int ks = 0; ks < kMlHidden / 16; ++ks) {
            const int k0 = 16 * ks + 8 * lk;
            split3(*(const float4*)&T[li][k0], *(const float4*)&T[li][k0 + 4], ah, am, al);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    mfma3(acc[a][nt], ah, am, al, ldb(&L.W2T[a][32 * nt + li][k0]));
        }
        wave_sync();
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int a = (s1m >> r) & 1;
                T[8 * (r >> 2) + 4 * lk + (r & 3)][32 * nt + li] =
                    (a ? acc[1][nt][r] : acc[0][nt][r]) * s1v[nt][r];
            }
        wave_sync();
        // dE/dG[c][f] = inv_sd[f] sum_k delta1[c][k] W1[k][f]
        f32x16 acc3[2][3];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int nt = 0; nt < 3; ++nt)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc3[a][nt][r] = 0.0f;
#pragma unroll
        for (int ks = 0; ks < kMlHidden / 16; ++ks) {
            const int k0 = 16 * ks + 8 * lk;
            split3(*(const float4*)&T[li][k0], *(const float4*)&T[li][k0 + 4], ah, am, al);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int nt = 0; nt < 3; ++nt)
                    mfma3(acc3[a][nt], ah, am, al, ldb(&L.W1T[a][32 * nt + li][k0]));
        }
#pragma unroll
        for (int nt = 0; nt < 3; ++nt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int q = 8 * (r >> 2) + 4 * lk + (r & 3), f = 32 * nt + li;
                const int a = (s1m >> r) & 1;
                if (q < nv)
                    R.ml_g[(size_t)(cbase + q) * kMlFeat + f] =
                        (a ? acc3[1][nt][r] : acc3[0][nt][r]) * L.isd[a][f];
            }
        wave_sync();  // the tile is reused by the next tile of this wavefront
    }
}

// ------------------------------------------------------------ pair forces
// dE_i/dd_ij for the list entries of centre (i, s) within r_ml.  The entries
// in range are compacted first (ballot, LDS), so the lanes work on pairs
// that count; their slots are kept for the gather.
constexpr int kMaxStage = 512;  // in-range entries of one centre (<= maxml)
constexpr int kRadWin = 7;      // radial channels on each side of the nearest (pair forces)

template <typename T>
__global__ void __launch_bounds__(256) k_ml_pair(const RepDev* __restrict__ reps, const MlDev m,
                                                 const BlockEntry* __restrict__ blocks,
                                                 const StepRef sync)
{
    using T4 = typename V4T<T>::type;
    __shared__ float gs[4][kMlFeat];
    __shared__ float as[4][kMlAux];
    __shared__ float4 st[4][kMaxStage];   // staged d_ij (x, y, z), slot bits in .w
    const int lb = xcd_block();
    const BlockEntry be = blocks[lb];
    const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = be.atom0 + wave, s = be.group;
    if (i >= R.N) return;
    float4* __restrict__ stage = st[wave];
    const int N = R.N, P = R.P;
    const size_t cidx = (size_t)s * N + i;
    for (int f = lane; f < kMlFeat; f += 64) gs[wave][f] = R.ml_g[cidx * kMlFeat + f];
    for (int f = lane; f < kMlAux; f += 64) as[wave][f] = R.ml_aux[cidx * kMlAux + f];
    const T4* __restrict__ u = (const T4*)R.ub[step_index(sync).p];
    const T4* __restrict__ ent = (const T4*)R.ml_nb + (size_t)i * R.maxml;
    const T4 ui = u[(size_t)i * P + s];
    const int cnt = R.ml_nc[i];
    const float rc = m.r_cut;
    const float idr = 1.0f / m.dr;
    const float em2 = fexp(-2.0f * m.eta_r * m.dr * m.dr);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int n = 0;
    for (int k0 = 0; k0 < cnt; k0 += 64) {
        const int k = k0 + lane;
        bool hit = false;
        float dx = 0.f, dy = 0.f, dz = 0.f;
        if (k < cnt) {
            const T4 E = ent[k];
            const T4 Uj = u[(size_t)ebits<T>(E) * P + s];
            dx = (float)((Uj.x - ui.x) - E.x);
            dy = (float)((Uj.y - ui.y) - E.y);
            dz = (float)((Uj.z - ui.z) - E.z);
            hit = dx * dx + dy * dy + dz * dz < rc * rc;
        }
        const uint64_t mask = __ballot(hit);
        const int q = n + __popcll(mask & below);
        if (hit && q < kMaxStage) stage[q] = make_float4(dx, dy, dz, __int_as_float(k));
        n += __popcll(mask);
    }
    n = min(n, kMaxStage);
    int* __restrict__ in_slots = R.ml_in + cidx * R.maxml;
    if (lane == 0) R.ml_nin[cidx] = n;
    wave_sync();
    float4* __restrict__ out = (float4*)R.ml_fpair + cidx * R.maxml;
    for (int q = lane; q < n; q += 64) {
        const float4 D = stage[q];
        const int k = __float_as_int(D.w);
        const float dx = D.x, dy = D.y, dz = D.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const int b = R.species[ebits<T>(ent[k])];
        const float* __restrict__ g = gs[wave] + b * kMlFeatSp;
        const float* __restrict__ A = as[wave] + b * kMlAng * 9;
        const float r = __builtin_sqrtf(r2), ir = 1.0f / r;
        const float rx = dx * ir, ry = dy * ir, rz = dz * ir;
        const float ang = kPiF * r / rc;
        const float fc = 0.5f * (__cosf(ang) + 1.0f);
        const float dfc = -0.5f * kPiF / rc * __sinf(ang);
        // radial: dE/dr = sum_c g_c e_c (-2 eta (r - mu_c) f_c + f_c'), over the
        // channels within kRadWin spacings of r (the others are below
        // e^{-eta (kRadWin dr)^2} = e^{-24.5} of the nearest).  From the
        // nearest channel outwards, e_{c+-1} = e_c q and q changes by the
        // factor e^{-2 eta dr^2} per channel, so three exponentials serve all.
        float S0 = 0.f, S1 = 0.f;
        {
            const int cn = min(max((int)rintf((r - m.mu0) * idr), 0), kMlRad - 1);
            const float x0 = r - (m.mu0 + m.dr * cn);
            const float e0 = fexp(-m.eta_r * x0 * x0);
            const float b = 2.0f * m.eta_r * m.dr;
            const float h = m.eta_r * m.dr * m.dr;
            S0 = g[cn] * e0;
            S1 = S0 * x0;
            float eu = e0, qu = fexp(b * x0 - h), xu = x0;   // towards larger c
            float ed = e0, qd = fexp(-b * x0 - h), xd = x0;  // towards smaller c
#pragma unroll
            for (int k = 1; k <= kRadWin; ++k) {
                eu *= qu;
                qu *= em2;
                xu -= m.dr;
                ed *= qd;
                qd *= em2;
                xd += m.dr;
                const int cu = cn + k, cd = cn - k;
                const float gu = cu < kMlRad ? g[min(cu, kMlRad - 1)] * eu : 0.0f;
                const float gd = cd >= 0 ? g[max(cd, 0)] * ed : 0.0f;
                S0 += gu + gd;
                S1 += gu * xu + gd * xd;
            }
        }
        float dEdr = -2.0f * m.eta_r * fc * S1 + dfc * S0;
        float ox = 0.f, oy = 0.f, oz = 0.f;  // terms off the pair axis
#pragma unroll
        for (int k8 = 0; k8 < kMlAng; ++k8) {
            const float x = r - (m.nu0 + m.da * k8);
            const float ea = fexp(-m.eta_a * x * x);
            const float ps = ea * fc;
            const float dps = ea * (-2.0f * m.eta_a * x * fc + dfc);
            const float* a = A + k8 * 9;
            const float g1 = g[kMlRad + k8], g2 = g[kMlRad + kMlAng + k8];
            // l = 1: 2 [psi' (rhat.A1) rhat + psi/r (A1 - (rhat.A1) rhat)]
            const float p = rx * a[0] + ry * a[1] + rz * a[2];
            dEdr += 2.0f * g1 * dps * p;
            const float c1 = 2.0f * g1 * ps * ir;
            ox += c1 * (a[0] - p * rx);
            oy += c1 * (a[1] - p * ry);
            oz += c1 * (a[2] - p * rz);
            // l = 2: 2 [psi' q rhat + 2 psi/r (A2 rhat - q rhat)], q = rhat.A2.rhat
            const float vx = a[3] * rx + a[6] * ry + a[7] * rz;
            const float vy = a[6] * rx + a[4] * ry + a[8] * rz;
            const float vz = a[7] * rx + a[8] * ry + a[5] * rz;
            const float qq = rx * vx + ry * vy + rz * vz;
            dEdr += 2.0f * g2 * dps * qq;
            const float c2 = 4.0f * g2 * ps * ir;
            ox += c2 * (vx - qq * rx);
            oy += c2 * (vy - qq * ry);
            oz += c2 * (vz - qq * rz);
        }
        out[k] = make_float4(dEdr * rx + ox, dEdr * ry + oy, dEdr * rz + oz, 0.0f);
        in_slots[q] = k;
    }
}

// F_i = sum over the entries in range (d_ij is exactly -d_ji, so both sides
// agree on which they are) of dE_i/dd_ij - dE_j/dd_ji, in list order, then
// the same closing kick / sampling as the pair kernel.  Blocks: the pair
// kernel's table (apb atoms, G beads per wavefront).
template <typename T, int G>
__global__ void __launch_bounds__(256) k_ml_gather(const RepDev* __restrict__ reps,
                                                   const MlDev m,
                                                   const BlockEntry* __restrict__ blocks,
                                                   int32_t flags, double* __restrict__ partials,
                                                   int apb)
{
    using T4 = typename V4T<T>::type;
    constexpr int NCH = 64 / G;
    __shared__ double red[4][kNobs];
    const int lb = xcd_block();
    const BlockEntry be = blocks[lb];
    const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bl = lane % G, ch = lane / G;
    const int i = be.atom0 + wave;
    const int N = R.N, P = R.P;
    const int s = be.group * G + bl;
    const bool active = wave < apb && i < N && s < P;
    double* const vrec = recorder_row(R, flags);
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (active) {
        const T4* __restrict__ ent = (const T4*)R.ml_nb + (size_t)i * R.maxml;
        const int* __restrict__ rev = R.ml_rev + (size_t)i * R.maxml;
        const float4* __restrict__ fp = (const float4*)R.ml_fpair;
        const size_t c = (size_t)s * N + i;
        const int* __restrict__ in_slots = R.ml_in + c * R.maxml;
        const int n = R.ml_nin[c];
        for (int q = ch; q < n; q += NCH) {
            const int k = in_slots[q];
            const int j = ebits<T>(ent[k]);
            const float4 a = fp[c * R.maxml + k];
            const float4 b = fp[((size_t)s * N + j) * R.maxml + rev[k]];
            fx += (double)(a.x - b.x);
            fy += (double)(a.y - b.y);
            fz += (double)(a.z - b.z);
        }
    }
#pragma unroll
    for (int off = G; off < 64; off <<= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
        fz += __shfl_xor(fz, off);
    }
    double ob[kNobs] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (active && lane < G) {
        const int spi = R.species[i];
        const size_t c = (size_t)s * N + i;
        const double e_atom = (double)R.ml_y[c] + m.e0[spi];
        const double f[3] = {fx, fy, fz};
        force_epilogue<T>(R, i, s, spi, f, e_atom, flags, ob, vrec);
    }
    if (flags & kSample) {
#pragma unroll
        for (int q = 0; q < kNobs; ++q) {
            double t = ob[q];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
            if (lane == 0) red[wave][q] = t;
        }
        __syncthreads();
        if (threadIdx.x < kNobs) {
            const double t = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                             red[3][threadIdx.x];
            partials[(size_t)lb * kNobs + threadIdx.x] = t;
        }
    }
}

// --------------------------------------------------------------- training
// One block per replica (frames of one bead): E_f = sum eatom, the loss
// w_E / B (dE / N)^2 + w_F / (3 N_tot) sum |dF|^2, dL/dF into ml_u and
// dL/dE_f into ml_ebar.
__global__ void __launch_bounds__(256) k_ml_loss(const RepDev* __restrict__ reps, int n_rep,
                                                 const double* __restrict__ eref,
                                                 const double* __restrict__ fref,
                                                 const int64_t* __restrict__ fref_off, double w_E,
                                                 double w_F, double n_tot,
                                                 double* __restrict__ loss_parts)
{
    __shared__ double red[4][2];
    const int r = blockIdx.x;
    const RepDev& R = reps[r];
    const int N = R.N;
    const double* __restrict__ fo = fref + fref_off[r];
    const float* __restrict__ F = (const float*)R.force;
    const double cF = 2.0 * w_F / (3.0 * n_tot);
    double e = 0.0, d2 = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        e += R.eatom[i];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double d = (double)F[(size_t)a * N + i] - fo[(size_t)a * N + i];
            d2 += d * d;
            R.ml_u[(size_t)a * N + i] = (float)(cF * d);
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        e += __shfl_xor(e, off);
        d2 += __shfl_xor(d2, off);
    }
    if (lane == 0) {
        red[wave][0] = e;
        red[wave][1] = d2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double E = 0.0, D2 = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            E += red[w][0];
            D2 += red[w][1];
        }
        const double dE = E - eref[r];
        loss_parts[r] = w_E / n_rep * (dE / N) * (dE / N) + w_F / (3.0 * n_tot) * D2;
        *R.ml_ebar = 2.0 * w_E / n_rep * dE / ((double)N * N);
    }
}

// v_i = sum_j (dG_i/dd_ij) (u_j - u_i): the descriptors' derivative along dL/dF.
template <typename T>
__global__ void __launch_bounds__(256) k_ml_jvp(const RepDev* __restrict__ reps, const MlDev m,
                                                const BlockEntry* __restrict__ blocks,
                                                const StepRef sync)
{
    using T4 = typename V4T<T>::type;
    __shared__ PairStage stage[4];
    const BlockEntry be = blocks[blockIdx.x];
    const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = be.atom0 + wave, s = be.group;
    if (i >= R.N) return;
    PairStage& st = stage[wave];
    const int N = R.N, P = R.P;
    const size_t cidx = (size_t)s * N + i;
    const T4* __restrict__ u = (const T4*)R.ub[step_index(sync).p];
    const T4 ui = u[(size_t)i * P + s];
    const float* __restrict__ uu = R.ml_u + (size_t)s * 3 * N;
    const float wix = uu[i], wiy = uu[N + i], wiz = uu[2 * N + i];
    const int cnt = R.ml_nc[i];
    const int c = lane & 31, h = lane >> 5;
    const int ka = lane & 7, qa = lane >> 3;
    const float mu_c = m.mu0 + m.dr * c;
    const float nu_k = m.nu0 + m.da * ka;
    float A[2][9];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int z = 0; z < 9; ++z) A[b][z] = R.ml_aux[cidx * kMlAux + (b * kMlAng + ka) * 9 + z];
    float v0 = 0.f, v1 = 0.f;                 // radial, per species
    float l1[2] = {0.f, 0.f}, l2[2] = {0.f, 0.f};
    for (int k0 = 0; k0 < cnt; k0 += 64) {
        const int n = stage_pairs<T, true>(R, m, i, s, ui, k0, cnt, st, lane, wix, wiy, wiz, u);
        for (int t = h; t < n; t += 2) {
            const float x = st.r[t] - mu_c;
            const float e = fexp(-m.eta_r * x * x);
            const float dph = e * (-2.0f * m.eta_r * x * st.fc[t] + st.dfc[t]);
            const float rw = st.rx[t] * st.wx[t] + st.ry[t] * st.wy[t] + st.rz[t] * st.wz[t];
            const bool b1 = st.sp[t] != 0.0f;
            v0 += b1 ? 0.0f : dph * rw;
            v1 += b1 ? dph * rw : 0.0f;
        }
        for (int t = qa; t < n; t += 8) {
            const float x = st.r[t] - nu_k;
            const float ea = fexp(-m.eta_a * x * x);
            const float ps = ea * st.fc[t];
            const float dps = ea * (-2.0f * m.eta_a * x * st.fc[t] + st.dfc[t]);
            const float rx = st.rx[t], ry = st.ry[t], rz = st.rz[t];
            const float wx = st.wx[t], wy = st.wy[t], wz = st.wz[t];
            const float ir = 1.0f / st.r[t];
            const float rw = rx * wx + ry * wy + rz * wz;
            const int b = st.sp[t] != 0.0f ? 1 : 0;
            float val1, val2;
            {
                const float* a = A[0];
                const float* a1b = A[1];
                const float p0 = rx * a[0] + ry * a[1] + rz * a[2];
                const float p1 = rx * a1b[0] + ry * a1b[1] + rz * a1b[2];
                const float aw0 = wx * a[0] + wy * a[1] + wz * a[2];
                const float aw1 = wx * a1b[0] + wy * a1b[1] + wz * a1b[2];
                const float p = b ? p1 : p0, aw = b ? aw1 : aw0;
                val1 = 2.0f * (dps * rw * p + ps * ir * (aw - rw * p));
                float M[6];
#pragma unroll
                for (int z = 0; z < 6; ++z) M[z] = b ? A[1][3 + z] : A[0][3 + z];
                const float vx = M[0] * rx + M[3] * ry + M[4] * rz;
                const float vy = M[3] * rx + M[1] * ry + M[5] * rz;
                const float vz = M[4] * rx + M[5] * ry + M[2] * rz;
                const float qq = rx * vx + ry * vy + rz * vz;
                const float vw = vx * wx + vy * wy + vz * wz;
                val2 = 2.0f * (dps * qq * rw + 2.0f * ps * ir * (vw - qq * rw));
            }
            l1[0] += b ? 0.0f : val1;
            l1[1] += b ? val1 : 0.0f;
            l2[0] += b ? 0.0f : val2;
            l2[1] += b ? val2 : 0.0f;
        }
        wave_sync();
    }
    v0 += __shfl_xor(v0, 32);
    v1 += __shfl_xor(v1, 32);
#pragma unroll
    for (int off = 8; off < 64; off <<= 1) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            l1[b] += __shfl_xor(l1[b], off);
            l2[b] += __shfl_xor(l2[b], off);
        }
    }
    float* __restrict__ v = R.ml_v + cidx * kMlFeat;
    if (lane < 32) {
        v[lane] = v0;
        v[kMlFeatSp + lane] = v1;
    }
    if (lane < 8) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            v[b * kMlFeatSp + kMlRad + lane] = l1[b];
            v[b * kMlFeatSp + kMlRad + kMlAng + lane] = l2[b];
        }
    }
}

// Forward (primal and tangent along xd = v inv_sd) and reverse mode of
// e_bar E_i - dE_i/dx . xd for one centre per wavefront; writes the rows the
// weight-gradient sums need.
__global__ void __launch_bounds__(1024) k_ml_train_mlp(const RepDev* __restrict__ reps,
                                                       const MlDev m,
                                                       const BlockEntry* __restrict__ blocks,
                                                       int n_blocks)
{
    extern __shared__ float4 lds_raw[];
    MlpLds& L = *reinterpret_cast<MlpLds*>(lds_raw);
    float* scratch = reinterpret_cast<float*>(reinterpret_cast<char*>(lds_raw) + sizeof(MlpLds));
    load_weights(L, m);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float* X = scratch + wave * (4 * kMlFeat);  // x[96], xd[96], then hidden vectors
    float* XD = X + kMlFeat;
    float* HA = X + 2 * kMlFeat;                // 64
    float* HB = HA + kMlHidden;                 // 64
    for (int b = blockIdx.x; b < n_blocks; b += gridDim.x) {
        const BlockEntry be = blocks[b];
        const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
        const int N = R.N;
        const double ebar = *R.ml_ebar;
        for (int q = wave; q < be.group; q += kMlpWaves) {
            const size_t c = (size_t)be.atom0 + q;
            const int a = R.species[c % N];
            for (int f = lane; f < kMlFeat; f += 64) {
                X[f] = (R.ml_G[c * kMlFeat + f] - L.mu[a][f]) * L.isd[a][f];
                XD[f] = R.ml_v[c * kMlFeat + f] * L.isd[a][f];
            }
            wave_sync();
            const int o = lane;
            float z1 = L.b1[a][o], z1d = 0.f;
            for (int f = 0; f < kMlFeat; ++f) {
                const float w = L.W1[a][o][f];
                z1 += w * X[f];
                z1d += w * XD[f];
            }
            const float sg1 = sigm(z1);
            const float h1 = z1 * sg1;
            const float s1 = sg1 * (1.0f + z1 * (1.0f - sg1));
            const float t1 = sg1 * (1.0f - sg1) * (2.0f + z1 * (1.0f - 2.0f * sg1));
            const float h1d = s1 * z1d;
            HA[o] = h1;
            HB[o] = h1d;
            wave_sync();
            float z2 = L.b2[a][o], z2d = 0.f;
            for (int k = 0; k < kMlHidden; ++k) {
                const float w = L.W2[a][o][k];
                z2 += w * HA[k];
                z2d += w * HB[k];
            }
            const float sg2 = sigm(z2);
            const float h2 = z2 * sg2;
            const float s2 = sg2 * (1.0f + z2 * (1.0f - sg2));
            const float t2 = sg2 * (1.0f - sg2) * (2.0f + z2 * (1.0f - 2.0f * sg2));
            const float h2d = s2 * z2d;
            const float w3 = L.w3[a][o];
            const float e = (float)ebar, om = -1.0f;
            const float z2b = e * w3 * s2 + om * w3 * t2 * z2d;
            const float z2db = om * w3 * s2;
            float* row = R.ml_adj + c * kMlAdj;
            // rows: xd[96] z1b z1db h1 h1d z2b z2db t3 e
            row[96 + 4 * 64 + o] = z2b;
            row[96 + 5 * 64 + o] = z2db;
            row[96 + 6 * 64 + o] = e * h2 + om * h2d;
            row[96 + 2 * 64 + o] = h1;
            row[96 + 3 * 64 + o] = h1d;
            wave_sync();  // HA / HB reads done
            HA[o] = z2b;
            HB[o] = z2db;
            wave_sync();
            float h1b = 0.f, h1db = 0.f;  // lane = k
            for (int oo = 0; oo < kMlHidden; ++oo) {
                const float w = L.W2[a][oo][lane];
                h1b += w * HA[oo];
                h1db += w * HB[oo];
            }
            row[96 + lane] = h1b * s1 + h1db * t1 * z1d;
            row[96 + 64 + lane] = h1db * s1;
            for (int f = lane; f < kMlFeat; f += 64) row[f] = XD[f];
            if (lane == 0) row[96 + 7 * 64] = e;
            wave_sync();  // X, XD, HA, HB are reused by the next centre
        }
    }
}

// dL/dtheta as outer-product sums over the centres of each species:
//   W1 += z1b x^T + z1db xd^T, W2 += z2b h1^T + z2db h1d^T, b1 += z1b,
//   b2 += z2b, w3 += t3, b3 += e.
// The two weight sums are dense contractions over the centres, run on the
// matrix cores: v_mfma_f32_32x32x2_f32 with A = (z_b, z_db) of one centre
// (its two columns) and B = (x, x_d) (its two rows), so one instruction adds
// both rank-one terms of a centre to a 32 x 32 tile, FP32 products (exact)
// and FP32 accumulation.  Workgroup g (8 wavefronts) takes the network tiles
// g, g + kWgBlocks, ... in order and stages 16 centres at a time in LDS
// (32 threads per centre, 16-byte loads; zeros for padding); wavefronts 0-3 accumulate species 0, 4-7 species 1
// (a centre of the other species enters as zeros): W1 (64 x 96) is 2 x 3
// tiles, W2 (64 x 64) 2 x 2, so wavefront w % 4 holds W1 row tile w % 4
// (w % 4 < 2: three column tiles) or W2 row tile w % 4 - 2 (two).  The bias
// sums stay on the vector ALU.  Partial sums go to part[g][a];
// k_ml_wgrad_sum adds the kWgBlocks partials in order in FP64.
constexpr int kWgStage = 16;
static_assert(kMlFeat == 96 && kMlHidden == 64, "the weight-gradient tiles assume 96 x 64 x 64");

struct __attribute__((aligned(16))) WgLds {
    float x[kWgStage][kMlFeat], xd[kWgStage][kMlFeat];
    float z1b[kWgStage][kMlHidden], z1db[kWgStage][kMlHidden];
    float h1[kWgStage][kMlHidden], h1d[kWgStage][kMlHidden];
    float z2b[kWgStage][kMlHidden], z2db[kWgStage][kMlHidden], t3[kWgStage][kMlHidden];
    float e[kWgStage];
    int sp[kWgStage];   // species of the centre, -1 for padding
};
static_assert(offsetof(WgLds, t3) - offsetof(WgLds, z1b) ==
                  6 * sizeof(float) * kWgStage * kMlHidden,
              "the seven adjoint blocks are consecutive in the stage");
static_assert(offsetof(WgLds, z1b) % 16 == 0 && offsetof(WgLds, xd) % 16 == 0,
              "16-byte stage stores");
static_assert(kWgStage * 32 == 512, "32 threads per staged centre");

__global__ void __launch_bounds__(512) k_ml_wgrad_part(const RepDev* __restrict__ reps,
                                                       const MlDev m,
                                                       const BlockEntry* __restrict__ blocks,
                                                       int n_blocks, float* __restrict__ part)
{
    __shared__ WgLds L;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int a = wave >> 2, role = wave & 3;          // species, tile role
    const int li = lane & 31, lk = lane >> 5;
    const bool w1role = role < 2;
    const int o0 = 32 * (w1role ? role : role - 2);   // output row tile
    f32x16 acc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
    // bias sums: threads of wavefront 0 (species 0) and 4 (species 1)
    float vb1 = 0.f, vb2 = 0.f, vw3 = 0.f, vb3 = 0.f;
    for (int b = blockIdx.x; b < n_blocks; b += gridDim.x) {
        const BlockEntry be = blocks[b];
        const RepDev& R = reps[be.rep];
        const int N = R.N;
        for (int q0 = 0; q0 < be.group; q0 += kWgStage) {
            __syncthreads();  // previous stage consumed
            {
                // 32 threads per centre, 16-byte loads along its rows
                const int qi = t >> 5, sub = t & 31;
                const int q = q0 + qi;
                const bool valid = q < be.group;
                const size_t c = (size_t)be.atom0 + (valid ? q : 0);
                const int sp = valid ? R.species[c % N] : -1;
                if (sub == 0) L.sp[qi] = sp;
                const float4* G4 = (const float4*)(R.ml_G + c * kMlFeat);
                const float4* row4 = (const float4*)(R.ml_adj + c * kMlAdj);
                const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
                if (sub < kMlFeat / 4) {
                    float4 g = valid ? G4[sub] : z4;
                    if (valid) {
                        const float* mu = m.mu + sp * kMlFeat + 4 * sub;
                        const float* is = m.inv_sd + sp * kMlFeat + 4 * sub;
                        g.x = (g.x - mu[0]) * is[0];
                        g.y = (g.y - mu[1]) * is[1];
                        g.z = (g.z - mu[2]) * is[2];
                        g.w = (g.w - mu[3]) * is[3];
                    }
                    *(float4*)&L.x[qi][4 * sub] = g;
                    *(float4*)&L.xd[qi][4 * sub] = valid ? row4[sub] : z4;
                }
                // z1b z1db h1 h1d z2b z2db t3: consecutive [kWgStage][64] arrays,
                // the adjoint row's blocks in the same order
                float* blk0 = &L.z1b[0][0];
                for (int k4 = sub; k4 < 7 * kMlHidden / 4; k4 += 32) {
                    const int blk = k4 / (kMlHidden / 4), o4 = k4 % (kMlHidden / 4);
                    *(float4*)(blk0 + ((size_t)blk * kWgStage + qi) * kMlHidden + 4 * o4) =
                        valid ? row4[kMlFeat / 4 + k4] : z4;
                }
                if (sub == 0) L.e[qi] = valid ? R.ml_adj[c * kMlAdj + kMlFeat + 7 * kMlHidden] : 0.0f;
            }
            __syncthreads();
            for (int qi = 0; qi < kWgStage; ++qi) {
                const bool mine = L.sp[qi] == a;   // uniform over the wavefront
                if (!mine) continue;
                if (w1role) {
                    const float av = lk ? L.z1db[qi][o0 + li] : L.z1b[qi][o0 + li];
#pragma unroll
                    for (int ft = 0; ft < 3; ++ft) {
                        const float bv = lk ? L.xd[qi][32 * ft + li] : L.x[qi][32 * ft + li];
                        acc[ft] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[ft], 0, 0, 0);
                    }
                } else {
                    const float av = lk ? L.z2db[qi][o0 + li] : L.z2b[qi][o0 + li];
#pragma unroll
                    for (int ht = 0; ht < 2; ++ht) {
                        const float bv = lk ? L.h1d[qi][32 * ht + li] : L.h1[qi][32 * ht + li];
                        acc[ht] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[ht], 0, 0, 0);
                    }
                }
                if (role == 0) {
                    vb1 += L.z1b[qi][lane];
                    vb2 += L.z2b[qi][lane];
                    vw3 += L.t3[qi][lane];
                    if (lane == 0) vb3 += L.e[qi];
                }
            }
        }
    }
    float* out = part + ((size_t)blockIdx.x * kMlSpecies + a) * kMlParamsSp;
    if (w1role) {
#pragma unroll
        for (int ft = 0; ft < 3; ++ft)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int o = o0 + 8 * (r >> 2) + 4 * lk + (r & 3);
                out[kMlOffW1 + o * kMlFeat + 32 * ft + li] = acc[ft][r];
            }
    } else {
#pragma unroll
        for (int ht = 0; ht < 2; ++ht)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int o = o0 + 8 * (r >> 2) + 4 * lk + (r & 3);
                out[kMlOffW2 + o * kMlHidden + 32 * ht + li] = acc[ht][r];
            }
    }
    if (role == 0) {
        out[kMlOffB1 + lane] = vb1;
        out[kMlOffB2 + lane] = vb2;
        out[kMlOffW3 + lane] = vw3;
        if (lane == 0) out[kMlOffB3] = vb3;
    }
}

// Sum of the n_part partial gradients in a fixed order, in FP64: block of 8
// wavefronts per 64 parameters, wavefront w adds partials
// [w n_part / 8, (w + 1) n_part / 8) in order, then the eight wavefront sums
// are added in order.
__global__ void __launch_bounds__(512) k_ml_wgrad_sum(const float* __restrict__ part, int n_part,
                                                      float* __restrict__ grad)
{
    __shared__ double ws[8][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (p < kMlParams) {
        const int a = p / kMlParamsSp, off = p % kMlParamsSp;
        const int g0 = (w * n_part) / 8, g1 = ((w + 1) * n_part) / 8;
        for (int g = g0; g < g1; ++g)
            acc += (double)part[((size_t)g * kMlSpecies + a) * kMlParamsSp + off];
    }
    ws[w][lane] = acc;
    __syncthreads();
    if (w == 0 && p < kMlParams) {
        double s = 0.0;
        for (int q = 0; q < 8; ++q) s += ws[q][lane];
        grad[p] = (float)s;
    }
}

__global__ void k_ml_adam(float* __restrict__ master, uint16_t* __restrict__ wq,
                          float* __restrict__ m1, float* __restrict__ m2,
                          const float* __restrict__ grad, int n, float lr, float b1, float b2,
                          float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float g = grad[p];
    const float a = b1 * m1[p] + (1.0f - b1) * g;
    const float v = b2 * m2[p] + (1.0f - b2) * g * g;
    m1[p] = a;
    m2[p] = v;
    const float w = master[p] - lr * (a / c1) / (sqrtf(v / c2) + eps);
    master[p] = w;
    wq[p] = to_bf16(w);
}

__global__ void k_ml_round(const float* __restrict__ master, uint16_t* __restrict__ wq, int n)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) wq[p] = to_bf16(master[p]);
}

// Sums of G and G^2 per (centre species, feature), and centre counts:
// stats [2][96][2] then [2] (FP64).  One workgroup per (species, feature):
// thread t takes centres t, t + 256, ... of every replica in order, then a
// fixed tree in LDS.
__global__ void __launch_bounds__(256) k_ml_stats(const RepDev* __restrict__ reps, int n_rep,
                                                  double* __restrict__ stats)
{
    __shared__ double red[3][256];
    const int a = blockIdx.x / kMlFeat, f = blockIdx.x % kMlFeat;
    double s1 = 0.0, s2 = 0.0, n = 0.0;
    for (int r = 0; r < n_rep; ++r) {
        const RepDev& R = reps[r];
        const size_t nc = (size_t)R.P * R.N;
        for (size_t c = threadIdx.x; c < nc; c += blockDim.x) {
            if (R.species[c % R.N] != a) continue;
            const double g = R.ml_G[c * kMlFeat + f];
            s1 += g;
            s2 += g * g;
            n += 1.0;
        }
    }
    red[0][threadIdx.x] = s1;
    red[1][threadIdx.x] = s2;
    red[2][threadIdx.x] = n;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        stats[(a * kMlFeat + f) * 2 + 0] = red[0][0];
        stats[(a * kMlFeat + f) * 2 + 1] = red[1][0];
        if (f == 0) stats[2 * kMlFeat * 2 + a] = red[2][0];
    }
}

size_t mfma_lds_bytes() { return sizeof(MfmaLds) + sizeof(float) * 32 * kTS * kMfmaWaves; }
size_t train_lds_bytes() { return sizeof(MlpLds) + sizeof(float) * kMlpWaves * 4 * kMlFeat; }

// Dynamic LDS above the default limit; once per kernel (done is the caller's flag).
template <typename K>
void allow_lds(K kernel, size_t bytes, bool& done)
{
    if (!done) {
        (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)bytes);
        done = true;
    }
}

}  // namespace

void launch_ml_lists(hipStream_t st, bool fp64, const RepDev* reps, const BlockEntry* nl_blocks,
                     int n_nl, int32_t* status, StepRef sync)
{
    const int grid = n_nl < 256 ? n_nl : 256;
    if (grid <= 0) return;
    if (fp64) {
        launch(k_ml_list<double>, dim3(grid), dim3(256), 0, st, reps, nl_blocks, n_nl, status, sync);
        launch(k_ml_rev<double>, dim3(n_nl), dim3(256), 0, st, reps, nl_blocks, n_nl, status, sync);
    } else {
        launch(k_ml_list<float>, dim3(grid), dim3(256), 0, st, reps, nl_blocks, n_nl, status, sync);
        launch(k_ml_rev<float>, dim3(n_nl), dim3(256), 0, st, reps, nl_blocks, n_nl, status, sync);
    }
}

void launch_ml_forward(hipStream_t st, bool fp64, const RepDev* reps, const MlDev& m,
                       const BlockEntry* cblocks, int n_cblocks, const BlockEntry* mblocks,
                       int n_mblocks, int n_rep, int32_t* status, StepRef sync)
{
    if (n_cblocks <= 0) return;
    const size_t lds = mfma_lds_bytes();
    static bool lds_set = false;
    allow_lds(k_ml_mlp_mfma, lds, lds_set);
    const int tiles4 = (2 * n_mblocks + kMfmaWaves - 1) / kMfmaWaves;
    const int mgrid = tiles4 < 256 ? tiles4 : 256;
    if (fp64) {
        launch(k_ml_desc<double>, dim3(n_cblocks), dim3(256), 0, st, reps, m, cblocks,
               n_rep, status, sync);
        launch(k_ml_mlp_mfma, dim3(mgrid), dim3(256), (uint32_t)lds, st, reps, m, mblocks,
               n_mblocks);
        launch(k_ml_pair<double>, dim3(n_cblocks), dim3(256), 0, st, reps, m, cblocks, sync);
    } else {
        launch(k_ml_desc<float>, dim3(n_cblocks), dim3(256), 0, st, reps, m, cblocks,
               n_rep, status, sync);
        launch(k_ml_mlp_mfma, dim3(mgrid), dim3(256), (uint32_t)lds, st, reps, m, mblocks,
               n_mblocks);
        launch(k_ml_pair<float>, dim3(n_cblocks), dim3(256), 0, st, reps, m, cblocks, sync);
    }
}

template <typename T>
static void gather_T(hipStream_t st, int G, const RepDev* reps, const MlDev& m,
                     const BlockEntry* blocks, int n_blocks, int32_t flags, double* partials,
                     int apb)
{
    const dim3 g(n_blocks), b(256);
    switch (G) {
    case 1: launch((k_ml_gather<T, 1>), g, b, 0, st, reps, m, blocks, flags, partials, apb); break;
    case 2: launch((k_ml_gather<T, 2>), g, b, 0, st, reps, m, blocks, flags, partials, apb); break;
    case 4: launch((k_ml_gather<T, 4>), g, b, 0, st, reps, m, blocks, flags, partials, apb); break;
    case 8: launch((k_ml_gather<T, 8>), g, b, 0, st, reps, m, blocks, flags, partials, apb); break;
    default: break;
    }
}

void launch_ml_gather(hipStream_t st, bool fp64, int G, int apb, const RepDev* reps,
                      const MlDev& m, const BlockEntry* blocks, int n_blocks, int32_t flags,
                      double* partials)
{
    if (n_blocks <= 0) return;
    if (fp64) gather_T<double>(st, G, reps, m, blocks, n_blocks, flags, partials, apb);
    else gather_T<float>(st, G, reps, m, blocks, n_blocks, flags, partials, apb);
}

void launch_ml_loss(hipStream_t st, const RepDev* reps, int n_rep, const double* eref,
                    const double* fref, const int64_t* fref_off, double w_E, double w_F,
                    double n_atoms_total, double* loss_parts)
{
    launch(k_ml_loss, dim3(n_rep), dim3(256), 0, st, reps, n_rep, eref, fref, fref_off, w_E, w_F,
           n_atoms_total, loss_parts);
}

void launch_ml_jvp(hipStream_t st, bool fp64, const RepDev* reps, const MlDev& m,
                   const BlockEntry* cblocks, int n_cblocks, StepRef sync)
{
    if (n_cblocks <= 0) return;
    if (fp64) launch(k_ml_jvp<double>, dim3(n_cblocks), dim3(256), 0, st, reps, m, cblocks, sync);
    else launch(k_ml_jvp<float>, dim3(n_cblocks), dim3(256), 0, st, reps, m, cblocks, sync);
}

void launch_ml_train_mlp(hipStream_t st, const RepDev* reps, const MlDev& m,
                         const BlockEntry* mblocks, int n_mblocks)
{
    if (n_mblocks <= 0) return;
    const size_t lds = train_lds_bytes();
    static bool lds_set = false;
    allow_lds(k_ml_train_mlp, lds, lds_set);
    const int grid = n_mblocks < 256 ? n_mblocks : 256;
    launch(k_ml_train_mlp, dim3(grid), dim3(1024), (uint32_t)lds, st, reps, m, mblocks, n_mblocks);
}

void launch_ml_wgrad(hipStream_t st, const RepDev* reps, const MlDev& m,
                     const BlockEntry* mblocks, int n_mblocks, float* part, float* grad)
{
    launch(k_ml_wgrad_part, dim3(kWgBlocks), dim3(512), 0, st, reps, m, mblocks, n_mblocks,
           part);
    launch(k_ml_wgrad_sum, dim3((kMlParams + 63) / 64), dim3(512), 0, st, part, (int)kWgBlocks,
           grad);
}

void launch_ml_adam(hipStream_t st, float* master, uint16_t* wq, float* mom1, float* mom2,
                    const float* grad, int n, float lr, float b1, float b2, float eps, float c1,
                    float c2)
{
    launch(k_ml_adam, dim3((n + 255) / 256), dim3(256), 0, st, master, wq, mom1, mom2, grad, n,
           lr, b1, b2, eps, c1, c2);
}

void launch_ml_round(hipStream_t st, const float* master, uint16_t* wq, int n)
{
    launch(k_ml_round, dim3((n + 255) / 256), dim3(256), 0, st, master, wq, n);
}

void launch_ml_stats(hipStream_t st, const RepDev* reps, int n_rep, double* stats)
{
    launch(k_ml_stats, dim3(2 * kMlFeat), dim3(256), 0, st, reps, n_rep, stats);
}

}  // namespace qtb
