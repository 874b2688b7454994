// forces.hip -- forces of every bead, the closing B(dt/2) kick, and the
// energy estimators.
//
// Each bead of the ring polymer feels the physical potential V (eq. 3-4;
// the 1/P factor is applied with the kick).  The pair potential is a
// Buckingham term in shifted-force form plus damped shifted force Coulomb
// (constants folded into PairParam; see qtb_internal.h).
//
// Mapping on CDNA4: W 64-wide wavefronts per atom i.  Lane l takes bead
// s = group*G + l % G and neighbour chunk l / G (+ 64/G per extra wavefront);
// the G beads of an atom share one neighbour list (built from bead
// centroids, entries hold the reference displacement, so a pair distance is
// d_ij + u_i - u_j with small u in the working precision).  Per-bead sums are
// reduced across chunks with wavefront shuffles and across the W wavefronts
// in LDS (FP64 accumulators): no atomics, no write conflicts.  The first
// lanes of the atom finish it: store the force, apply the kick, and on
// sampling steps form the eq. (5) terms.
#include "force_epilogue.h"
#include "qtb_internal.h"
#include "ring_step.h"

namespace qtb {
namespace {

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

__device__ __forceinline__ int32_t as_bits(float x) { return __float_as_int(x); }
__device__ __forceinline__ int32_t as_bits(double x) { return (int32_t)__double_as_longlong(x); }

__device__ __forceinline__ float t_exp(float x) { return expf(x); }
__device__ __forceinline__ double t_exp(double x) { return exp(x); }
__device__ __forceinline__ float t_erfc(float x) { return erfcf(x); }
__device__ __forceinline__ double t_erfc(double x) { return erfc(x); }
__device__ __forceinline__ float t_rsqrt(float x) { return rsqrtf(x); }
__device__ __forceinline__ double t_rsqrt(double x) { return 1.0 / sqrt(x); }

// Sum a value over all 64 lanes (result in every lane).
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) x += __shfl_xor(x, off);
    return x;
}

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
template <typename T> struct NV;
template <> struct NV<float> { using v4 = f4v; };
template <> struct NV<double> { using v4 = d4v; };
// Workspace pointers live in RepDev (generic address space); casting them to
// the global address space lets the compiler emit global (not flat) loads.
template <typename X>
using gptr = const __attribute__((address_space(1))) X*;

template <typename T> __device__ __forceinline__ T as_bits_t(int32_t b);
template <> __device__ __forceinline__ float as_bits_t<float>(int32_t b) { return __int_as_float(b); }
template <> __device__ __forceinline__ double as_bits_t<double>(int32_t b)
{
    return __longlong_as_double((long long)b);
}

__device__ __forceinline__ int32_t vbits(f4v x) { return __float_as_int(x.w); }
__device__ __forceinline__ int32_t vbits(d4v x) { return (int32_t)__double_as_longlong(x.w); }

// Positions of step n for the pair loop: relative coordinates u (current
// parity) measured from the list's references.  RECON: the lists were just
// rebuilt around the current centroids c, so a neighbour's relative position
// is rebuilt as (r_ref + u) - c from the previous references (all read-only
// while the kernel runs; the owners update their own data in place).
// POSREF: the lists were just rebuilt and the positions are read-only in
// this kernel: relative positions are (T)(r - c) from the FP64 positions, as
// the list kernel computes them.
enum PosMode { kPosDirect = 0, kPosRecon = 1, kPosRef = 2 };

template <typename T, int MODE>
struct PairPos {
    using V4 = typename NV<T>::v4;
    gptr<V4> u;
    gptr<double> rref, cen;
    int N, P;
    gptr<double> pos;
    gptr<int32_t> species;
    __device__ __forceinline__ V4 at(int j, int s) const
    {
        V4 v;
        if constexpr (MODE == kPosRef) {
            const size_t b = (size_t)s * 3 * N + j;
            v.x = (T)(pos[b] - cen[j]);
            v.y = (T)(pos[b + N] - cen[N + j]);
            v.z = (T)(pos[b + 2 * (size_t)N] - cen[2 * (size_t)N + j]);
            v.w = as_bits_t<T>(species[j]);
        } else {
            v = u[(size_t)j * P + s];
            if constexpr (MODE == kPosRecon) {
                const double x = (rref[j] + (double)v.x) - cen[j];
                const double y = (rref[N + j] + (double)v.y) - cen[N + j];
                const double z = (rref[2 * (size_t)N + j] + (double)v.z) - cen[2 * (size_t)N + j];
                v.x = (T)x;
                v.y = (T)y;
                v.z = (T)z;
            }
        }
        return v;
    }
};

// Buffer resource over [base, base + bytes) for raw buffer loads: 32-bit
// byte offsets instead of 64-bit address arithmetic, and loads past the end
// return zeros.  base and bytes must be uniform over the wavefront.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    const uint64_t a = (uint64_t)base;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const void* b = (const void*)(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(b), (short)0,
                                             (int)__builtin_amdgcn_readfirstlane(bytes),
                                             0x00020000);
}
__device__ __forceinline__ f4v bload(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}

// NS: species count rounded up to 2 or 4 (parameters of the centre atom's
// row are kept in registers and picked per neighbour with selects).
// FAST (FP32 only): hardware rsq / exp2, the Coulomb force shape
// erfc(x) + (2x/sqrt(pi)) e^{-x^2} = 1 + (r r^2) psi(s) as a polynomial of
// degree DEG in s = r^2 (2 / r_cut^2) - 1 (no exponential), and for the
// energy the fitted erfcx polynomial.
// Force (FP64 sums), if want_e the energy, and if want_w the pair virial
// sum F(r) r of bead
// s of atom i over its list: the core entries (reference distance below
// r_cut) at slots 0 .. core - 1, then the shell entries at slots maxnb - 1,
// maxnb - 2, ...; lane entries ch, ch + ST, ... of each range.  spi
// receives the atom's species.
template <typename T, int NS, bool FAST, int DEG, int MODE, int G>
__device__ __forceinline__ void pair_sum(const RepDev& R, const PairTable<T>& tab,
                                         const PairPos<T, MODE>& pp, int i, int s, int ch,
                                         int ST, bool want_e, bool want_w, double& fx,
                                         double& fy, double& fz, double& e, double& w, int& spi,
                                         double lscale, const f4v* ltab)
{
    using V4 = typename NV<T>::v4;
    const V4 ui = pp.at(i, s);
    spi = vbits(ui);
    const int row = __builtin_amdgcn_readfirstlane(spi) * kMaxSpecies;
    T pArho[NS], pirho[NS], pC6[NS], pkqq[NS], pF0[NS], pA[NS], pC[NS], pE0[NS];
#pragma unroll
    for (int b = 0; b < NS; ++b) {
        const PairParam<T>& q = tab.p[row + b];
        pArho[b] = q.Arho;
        pirho[b] = FAST ? q.irho2 : q.irho;
        pC6[b] = q.C6;
        pkqq[b] = q.kqq;
        pF0[b] = q.F0;
        pA[b] = q.A;
        pC[b] = q.C;
        pE0[b] = q.E0;
    }
    // FP32 path with several species: a neighbour's parameters come from the
    // block's LDS copy of the centre species' row (two 16-byte reads per
    // pair, indexed by the neighbour's species: no per-species registers and
    // no selects).  Otherwise keep the parameters of neighbour species 1,
    // 2, ... in VGPRs for the whole loop (an instruction on gfx950 reads at
    // most one SGPR, VCC included, so a select of a uniform species-0 value
    // needs its own move).
    constexpr bool LTAB = FAST && NS >= 2;
    const f4v* const lrow = LTAB ? ltab + 2 * row : nullptr;
    if constexpr (!LTAB) {
#pragma unroll
        for (int b = 1; b < NS; ++b) {
            asm volatile("" : "+v"(pArho[b]), "+v"(pirho[b]), "+v"(pC6[b]), "+v"(pkqq[b]),
                         "+v"(pF0[b]));
        }
    }
    T ex[DEG + 1], ph[DEG + 1];
#pragma unroll
    for (int k = 0; k <= DEG; ++k) {
        ex[k] = tab.ex[k];
        ph[k] = tab.ph[k];
    }
    const T rc2 = tab.rc2, a2l = tab.a2l, s_mul = tab.s_mul, alpha = tab.alpha, g = tab.g;
    const T ph_s = tab.ph_s;
    // the Horner start in a VGPR, so its first FMA reads one SGPR only
    T ph_top = ph[DEG];
    asm volatile("" : "+v"(ph_top));
    const int maxnb = R.maxnb;
    const int cnt = R.nb_count[i], ncore = R.nb_core[i];
    // entries of a list built before the box last changed scale with it,
    // by lscale (entries built in this pass, MODE kPosRef, have the current
    // geometry)
    const T lsc = (T)lscale;
    // FP32 path: the lane's pair virial in FP32 (one FMA per pair), added to
    // the FP64 sum once at the end (the pressure needs no more)
    float wf = 0.0f;

    auto pair = [&](const V4 E0, const V4 U0) {
        T dx, dy, dz;
        if constexpr (MODE == kPosRef) {
            dx = (E0.x + ui.x) - U0.x;
            dy = (E0.y + ui.y) - U0.y;
            dz = (E0.z + ui.z) - U0.z;
        } else if constexpr (sizeof(T) == 4) {  // lsc = 1: the same bits as E + u
            dx = __builtin_fmaf(E0.x, lsc, ui.x) - U0.x;
            dy = __builtin_fmaf(E0.y, lsc, ui.y) - U0.y;
            dz = __builtin_fmaf(E0.z, lsc, ui.z) - U0.z;
        } else {
            dx = __builtin_fma(E0.x, lsc, ui.x) - U0.x;
            dy = __builtin_fma(E0.y, lsc, ui.y) - U0.y;
            dz = __builtin_fma(E0.z, lsc, ui.z) - U0.z;
        }
        const T r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < rc2) {
            const int spj = vbits(U0);
            T Arho = pArho[0], irho = pirho[0], C6 = pC6[0], kqq = pkqq[0], F0 = pF0[0];
            f4v q1 = {0.0f, 0.0f, 0.0f, 0.0f};
            if constexpr (LTAB) {
                const f4v q0 = lrow[2 * spj];
                Arho = q0.x;
                irho = q0.y;
                C6 = q0.z;
                kqq = q0.w;
                if (want_e) {
                    q1 = lrow[2 * spj + 1];
                    F0 = q1.x;
                } else {
                    F0 = ((const float*)(lrow + 2 * spj + 1))[0];
                }
            } else {
#pragma unroll
                for (int b = 1; b < NS; ++b) {
                    const bool m = spj == b;
                    Arho = m ? pArho[b] : Arho;
                    irho = m ? pirho[b] : irho;
                    C6 = m ? pC6[b] : C6;
                    kqq = m ? pkqq[b] : kqq;
                    F0 = m ? pF0[b] : F0;
                }
            }
            T rinv, r, e1, ec = (T)0, e2 = (T)0, fr;
            if constexpr (FAST) {
                rinv = __builtin_amdgcn_rsqf(r2);
                r = r2 * rinv;
                e1 = __builtin_amdgcn_exp2f(-r * irho);
                const T sp = fmaf(r2, ph_s, -1.0f);
                T ps = ph_top;
#pragma unroll
                for (int k = DEG - 1; k >= 0; --k) ps = fmaf(ps, sp, ph[k]);
                // F / r = (Arho e1 + F0 + kqq / r^2) / r + kqq psi - C6 / r^8:
                // the Coulomb shape over r^3 is 1 / r^3 + psi(s)
                const T rinv2 = rinv * rinv;
                const T rinv4 = rinv2 * rinv2;
                T a = fmaf(Arho, e1, F0);
                a = fmaf(kqq, rinv2, a);
                const T c = fmaf(-C6, rinv4 * rinv4, kqq * ps);
                fr = fmaf(a, rinv, c);
                if (want_e) {
                    e2 = __builtin_amdgcn_exp2f(-r2 * a2l);
                    const T sx = fmaf(r, s_mul, -1.0f);
                    T pe = ex[DEG];
#pragma unroll
                    for (int k = DEG - 1; k >= 0; --k) pe = fmaf(pe, sx, ex[k]);
                    ec = e2 * pe;
                }
            } else {
                rinv = t_rsqrt(r2);
                r = r2 * rinv;
                e1 = t_exp(-r * irho);
                const T x = alpha * r;
                e2 = t_exp(-x * x);
                ec = t_erfc(x);
                const T Fc = ec * (rinv * rinv) + g * e2 * rinv;
                const T rinv2 = rinv * rinv;
                const T rinv6 = rinv2 * rinv2 * rinv2;
                fr = (Arho * e1 - C6 * rinv6 * rinv + kqq * Fc + F0) * rinv;
            }
            if constexpr (sizeof(T) == 4) {
                // FP64 sums of the exact products (fr dx in FP64): one
                // conversion of fr shared by the three components
                const double frd = (double)fr;
                fx = __builtin_fma(frd, (double)dx, fx);
                fy = __builtin_fma(frd, (double)dy, fy);
                fz = __builtin_fma(frd, (double)dz, fz);
            } else {
                fx += fr * dx;
                fy += fr * dy;
                fz += fr * dz;
            }
            if (want_e) {
                const T rinv2 = rinv * rinv;
                const T rinv6 = rinv2 * rinv2 * rinv2;
                T A = pA[0], C = pC[0], E0c = pE0[0];
                if constexpr (LTAB) {
                    A = q1.y;
                    C = q1.z;
                    E0c = q1.w;
                } else {
#pragma unroll
                    for (int b = 1; b < NS; ++b) {
                        const bool m = spj == b;
                        A = m ? pA[b] : A;
                        C = m ? pC[b] : C;
                        E0c = m ? pE0[b] : E0c;
                    }
                }
                e += (double)(A * e1 - C * rinv6 + kqq * ec * rinv - F0 * r + E0c);
            }
            if (want_w) {
                if constexpr (FAST) wf = fmaf(fr, r2, wf);
                else w += (double)(fr * r2);
            }
        }
    };

    if constexpr (MODE == kPosDirect && sizeof(T) == 4) {
        // buffer loads with 32-bit byte offsets: entry slot q of atom i at
        // 16 q, bead s of neighbour j at 16 (j P + s)
        const __amdgpu_buffer_rsrc_t re =
            make_rsrc((const char*)R.nb_entries + (size_t)i * maxnb * 16, (uint32_t)maxnb * 16);
        const __amdgpu_buffer_rsrc_t ru =
            make_rsrc((const void*)(uintptr_t)pp.u, (uint32_t)(R.N * R.P) * 16u);
        const uint32_t Pb = (uint32_t)R.P * 16u, sb = (uint32_t)s * 16u;
        // one range: n entries, lane entries k = ch, ch + ST, ... at slots
        // first + dir k; three-stage pipeline (entry k + 2 ST and the
        // neighbour of entry k + ST load while entry k is evaluated)
        auto uoff = [&](const f4v E) { return __umul24((uint32_t)vbits(E), Pb) + sb; };
        auto range = [&](int n, int first, int dir) {
            if (ch >= n) return;
            const uint32_t dstep = (uint32_t)(dir * ST * 16);
            uint32_t eo = (uint32_t)(first + dir * ch) * 16u;
            f4v E0 = bload(re, eo), E1 = bload(re, eo + dstep), E2;
            f4v U0 = bload(ru, uoff(E0)), U1;
            int k = ch;
            // unrolled six times so that the three entry and two neighbour
            // registers rotate by renaming instead of copies
#define QTB_PAIR_STEP(Ea, Eb, Ec, Ua, Ub)      \
    if (k >= n) break;                         \
    Ec = bload(re, eo + 2 * dstep);            \
    Ub = bload(ru, uoff(Eb));                  \
    pair(Ea, Ua);                              \
    eo += dstep;                               \
    k += ST;
            for (;;) {
                QTB_PAIR_STEP(E0, E1, E2, U0, U1)
                QTB_PAIR_STEP(E1, E2, E0, U1, U0)
                QTB_PAIR_STEP(E2, E0, E1, U0, U1)
                QTB_PAIR_STEP(E0, E1, E2, U1, U0)
                QTB_PAIR_STEP(E1, E2, E0, U0, U1)
                QTB_PAIR_STEP(E2, E0, E1, U1, U0)
            }
#undef QTB_PAIR_STEP
        };
        range(ncore, 0, 1);
        range(cnt - ncore, maxnb - 1, -1);
    } else {
        gptr<V4> ent = (gptr<V4>)R.nb_entries + (size_t)i * maxnb;
        auto range = [&](int n, int first, int dir) {
            if (ch >= n) return;
            auto slot = [&](int k) { return first + dir * (k < n ? k : 0); };
            int k = ch;
            V4 E0 = ent[slot(k)];
            V4 E1 = ent[slot(k + ST)];
            V4 U0 = pp.at(vbits(E0), s);
            while (k < n) {
                const V4 E2 = ent[slot(k + 2 * ST)];
                const V4 U1 = pp.at(vbits(E1), s);
                pair(E0, U0);
                E0 = E1;
                E1 = E2;
                U0 = U1;
                k += ST;
            }
        };
        range(ncore, 0, 1);
        range(cnt - ncore, maxnb - 1, -1);
    }
    if (FAST && want_w) w += (double)wf;
}

// The block's LDS copy of the pair parameters for the FP32 path with
// several species (see pair_sum): per species pair (Arho, irho2, C6, kqq)
// and (F0, A, C, E0).  The caller synchronises the block afterwards.
template <typename T, int NS, bool FAST>
__device__ __forceinline__ void fill_ltab(const PairTable<T>& tab, f4v* ltab)
{
    if constexpr (FAST && NS >= 2) {
        for (int t = threadIdx.x; t < kPairs; t += blockDim.x) {
            const PairParam<T>& q = tab.p[t];
            ltab[2 * t] = f4v{(float)q.Arho, (float)q.irho2, (float)q.C6, (float)q.kqq};
            ltab[2 * t + 1] = f4v{(float)q.F0, (float)q.A, (float)q.C, (float)q.E0};
        }
    }
}

// Lanes with the same bead: reduce across chunks (shuffles), then across the
// W wavefronts of the atom (LDS part[wave][bead][4]); the sums end in the
// lanes < G of the atom's first wavefront.
template <int G>
__device__ __forceinline__ void reduce_atom(double& fx, double& fy, double& fz, double& e,
                                            double& vir, bool want_e, bool want_w, int W,
                                            int wave, int wsub, int lane, double (*part)[G][5])
{
#pragma unroll
    for (int off = G; off < 64; off <<= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
        fz += __shfl_xor(fz, off);
        if (want_e) e += __shfl_xor(e, off);
        if (want_w) vir += __shfl_xor(vir, off);
    }
    if (W > 1) {
        if (lane < G) {
            part[wave][lane][0] = fx;
            part[wave][lane][1] = fy;
            part[wave][lane][2] = fz;
            part[wave][lane][3] = e;
            part[wave][lane][4] = vir;
        }
        __syncthreads();
        if (wsub == 0 && lane < G) {
            for (int w = 1; w < W; ++w) {
                fx += part[wave + w][lane][0];
                fy += part[wave + w][lane][1];
                fz += part[wave + w][lane][2];
                e += part[wave + w][lane][3];
                vir += part[wave + w][lane][4];
            }
        }
    }
}

// Block sums of the observable slots into partials[lb] (lb: the block's
// table entry).
__device__ __forceinline__ void block_partials(const double* ob, int wave, int lane, int lb,
                                               double (*red)[kNobs], double* partials)
{
#pragma unroll
    for (int q = 0; q < kNobs; ++q) {
        const double t = wave_sum(ob[q]);
        if (lane == 0) red[wave][q] = t;
    }
    __syncthreads();
    if (threadIdx.x < kNobs) {
        const double t = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                         red[3][threadIdx.x];
        partials[(size_t)lb * kNobs + threadIdx.x] = t;
    }
}

// Rebuild the list of atom i (one wavefront, all bead groups share it) from
// the current centroids c and spreads dev (read-only in this kernel): pairs
// within r_cut + skin + dev_i + dev_j, every periodic image, ballot-compacted
// in a fixed order.  All four wavefronts of the block help stage candidate
// tiles in LDS; only waves with active set list.
template <typename T>
__device__ void rebuild_list(const RepDev& R, int i, bool active, const double* cx,
                             const double* cy, const double* cz, const double* dv,
                             int32_t* status, double* tx, double* ty, double* tz, double* td,
                             double* dmax_s, double box_scale)
{
    using V4 = typename NV<T>::v4;
    const int N = R.N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double xi = 0.0, yi = 0.0, zi = 0.0, devi = 0.0;
    if (active) {
        xi = cx[i];
        yi = cy[i];
        zi = cz[i];
        devi = dv[i];
    }
    const double Lx = R.box[0] * box_scale, Ly = R.box[1] * box_scale, Lz = R.box[2] * box_scale;
    const double iLx = 1.0 / Lx, iLy = 1.0 / Ly, iLz = 1.0 / Lz;
    double dmax = 0.0;
    for (int j = threadIdx.x; j < N; j += 256) dmax = fmax(dmax, dv[j]);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) dmax = fmax(dmax, __shfl_xor(dmax, off));
    if (lane == 0) dmax_s[wave] = dmax;
    __syncthreads();
    dmax = fmax(fmax(dmax_s[0], dmax_s[1]), fmax(dmax_s[2], dmax_s[3]));
    const double Rmax = R.r_cs + devi + dmax;
    bool over = false;
    const int mx = image_range(Rmax, iLx, over), my = image_range(Rmax, iLy, over),
              mz = image_range(Rmax, iLz, over);
    if (over && active && lane == 0) atomicOr(status, kStatusRange);
    V4* __restrict__ ent = (V4*)R.nb_entries + (size_t)i * R.maxnb;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const double rc2 = R.r_cut * R.r_cut;
    int ncore = 0, nshell = 0;
    for (int t0 = 0; t0 < N; t0 += 256) {
        __syncthreads();
        const int jl = t0 + threadIdx.x;
        if (jl < N) {
            tx[threadIdx.x] = cx[jl];
            ty[threadIdx.x] = cy[jl];
            tz[threadIdx.x] = cz[jl];
            td[threadIdx.x] = dv[jl];
        }
        __syncthreads();
        if (!active) continue;
        const int tn = min(256, N - t0);
        for (int c0 = 0; c0 < tn; c0 += 64) {
            const int jj = c0 + lane;
            const int j = t0 + jj;
            const bool valid = jj < tn;
            const double Rij = R.r_cs + devi + (valid ? td[jj] : 0.0);
            const double R2 = Rij * Rij;
            double dx = 0.0, dy = 0.0, dz = 0.0;
            if (valid) {
                dx = xi - tx[jj];
                dy = yi - ty[jj];
                dz = zi - tz[jj];
                dx -= Lx * rint(dx * iLx);
                dy -= Ly * rint(dy * iLy);
                dz -= Lz * rint(dz * iLz);
            }
            for (int nx = -mx; nx <= mx; ++nx)
                for (int ny = -my; ny <= my; ++ny)
                    for (int nz = -mz; nz <= mz; ++nz) {
                        const double ex = dx + nx * Lx, ey = dy + ny * Ly, ez = dz + nz * Lz;
                        const double r2 = ex * ex + ey * ey + ez * ez;
                        const bool self = (j == i) && nx == 0 && ny == 0 && nz == 0;
                        const bool hit = valid && r2 < R2 && !self;
                        V4 v;
                        v.x = (T)ex;
                        v.y = (T)ey;
                        v.z = (T)ez;
                        v.w = as_bits_t<T>(j);
                        list_push(ent, R.maxnb, hit, r2 < rc2, v, below, ncore, nshell);
                    }
        }
    }
    if (active && lane == 0)
        list_finish(R.nb_count, R.nb_core, i, R.maxnb, ncore, nshell, status);
    __syncthreads();
}

// Occupancy targets (measured on the 4096-atom x P = 8 workload): the plain
// FP32 force pass at eight wavefronts per SIMD (64 registers, a few spilled)
// ran 27.9 us against 28.6 at five; the sampling pass keeps five without
// spills; FP64 is left to the compiler.
template <typename T, int G, int NS, bool FAST, int DEG, int EM>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 1 : (EM == 2 ? 5 : 7)))) k_force_pair(const RepDev* __restrict__ reps,
                                                    const BlockEntry* __restrict__ blocks,
                                                    const PairTable<T> tab, int32_t flags,
                                                    double* __restrict__ partials, int clear,
                                                    int n_rep, int32_t* __restrict__ status,
                                                    const StepRef sync, int W)
{
    using V4 = typename NV<T>::v4;
    using T4 = typename Vec4<T>::type;
    constexpr int NCH = 64 / G;   // neighbour chunks per wavefront
    // W wavefronts per atom (1, 2 or 4), 4 / W atoms per block
    __shared__ double part[4][G][5];
    __shared__ double red[4][kNobs];
    __shared__ double tx[256], ty[256], tz[256], td[256];
    __shared__ double dmax_s[4];
    const int lb = xcd_block();
    const BlockEntry be = blocks[lb];
    const int rep = __builtin_amdgcn_readfirstlane(be.rep);
    const RepDev& R = reps[rep];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = wave / W, wsub = wave % W;
    const int bl = lane % G, ch = lane / G + wsub * NCH;
    const int i = be.atom0 + slot;
    const int N = R.N, P = R.P;
    const bool active = i < N;
    const int s = be.group * G + bl;
    __shared__ f4v ltab[2 * kPairs];
    if constexpr (FAST && NS >= 2) {
        fill_ltab<T, NS, FAST>(tab, ltab);
        __syncthreads();
    }
    // energies and the pair virial only in the instantiation that samples or
    // evaluates (EM = 2: flags & (kSample | kEvaluate)), the pair virial alone
    // for a barostat's step (EM = 1: kPressure): the plain force pass keeps
    // fewer registers live
    constexpr bool want_e = EM == 2;
    constexpr bool want_w = EM >= 1;
    double* const vrec = recorder_row(R, flags);
    const StepIdx si = step_index(sync);
    // clear == 1: the list kernel ran before; this step's and the previous
    // step's flags are done.  clear == 2: rebuild the lists here if this step
    // flagged it (no list kernel); its flag stays set for the other
    // workgroups and is cleared by the next step's force pass.
    const bool rebuild = clear == 2 && R.rflag[si.f] != 0;  // uniform over the block
    if (blockIdx.x == 0 && clear) {
        const int fold = si.f == 0 ? 2 : si.f - 1;
        for (int r = threadIdx.x; r < n_rep; r += blockDim.x) {
            if (clear == 1) reps[r].rflag[si.f] = 0;
            reps[r].rflag[fold] = 0;
        }
        if (threadIdx.x == 0) {
            if (clear == 1) status[kAnyRebuild + si.f] = 0;
            status[kAnyRebuild + fold] = 0;
        }
    }
    const double* __restrict__ cen = R.cnb[si.p];
    // Within a step (kKick) the positions already carry a barostat's pending
    // box factor npt_sr, which the box and the lists' scale take at the end
    // of the step (k_barostat); between steps they agree as they are.
    const double bsc = (flags & kKick) ? R.npt_sr : 1.0;
    const double lscale = R.npt_S * bsc;
    if (rebuild) {
        rebuild_list<T>(R, i, active && wsub == 0, cen, cen + N, cen + 2 * (size_t)N,
                        R.devn[si.p], status, tx, ty, tz, td, dmax_s, bsc);
        if (active && wsub == 0) {
            // new references and relative positions of the atom, as the list kernel
            if (lane < 3) R.rrefb[si.p][(size_t)lane * N + i] = cen[(size_t)lane * N + i];
            if (lane == 0) R.devbb[si.p][i] = R.devn[si.p][i];
            const T spb = as_bits_t<T>(R.species[i]);
            for (int b = lane; b < P; b += 64) {
                T4 v;
                v.x = (T)(R.pos[((size_t)b * 3 + 0) * N + i] - cen[i]);
                v.y = (T)(R.pos[((size_t)b * 3 + 1) * N + i] - cen[N + i]);
                v.z = (T)(R.pos[((size_t)b * 3 + 2) * N + i] - cen[2 * (size_t)N + i]);
                v.w = spb;
                ((T4*)R.ub[si.p])[(size_t)i * P + b] = v;
            }
        }
    }
    double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0, vir = 0.0;
    int spi = 0;
    if (active) {
        if (rebuild) {
            const PairPos<T, kPosRef> pp{nullptr, nullptr, (gptr<double>)cen, N, P,
                                         (gptr<double>)R.pos, (gptr<int32_t>)R.species};
            pair_sum<T, NS, FAST, DEG, kPosRef, G>(R, tab, pp, i, s, ch, NCH * W, want_e, want_w,
                                                fx, fy, fz, e, vir, spi, 1.0, ltab);
        } else {
            // u is atom-major [N][P]: the G beads of a neighbour share cache lines
            const PairPos<T, kPosDirect> pp{(gptr<V4>)R.ub[si.p] + 0, nullptr, nullptr, N, P,
                                            nullptr, nullptr};
            pair_sum<T, NS, FAST, DEG, kPosDirect, G>(R, tab, pp, i, s, ch, NCH * W, want_e,
                                                   want_w, fx, fy, fz, e, vir, spi, lscale, ltab);
        }
    }
    reduce_atom<G>(fx, fy, fz, e, vir, want_e, want_w, W, wave, wsub, lane, part);
    double ob[kNobs] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (active && wsub == 0 && lane < G && s < P) {
        const double f[3] = {fx, fy, fz};
        force_epilogue<T>(R, i, s, spi, f, 0.5 * e, flags, ob, vrec);
        // each pair is listed from both sides
        if (flags & (kSample | kPressure)) ob[5] = 0.5 * vir;
    }
    if (flags & (kSample | kCompare | kPressure)) block_partials(ob, wave, lane, lb, red, partials);
}

// One step of the pair potential for P = G <= 8 beads (all beads of an atom
// in one wavefront), n = the step counter:
//   [rebuild the lists if step n flagged it] -> forces at x_n -> closing
//   half-kick of step n-1 (and its sampling) -> opening half-kick of step n
//   -> normal modes, A(dt/2) O(dt) A(dt/2) with zeta_row -> x_{n+1}.
// Neighbours read u, centroids and references of parity n & 1; the owner
// writes its atom's data for step n + 1 into parity (n + 1) & 1 and updates
// its positions and velocities in place.  Bit for bit the same arithmetic
// as the separate update and force kernels.
template <typename T, int G, int NS, bool FAST, int DEG, bool WE>
__global__ void __launch_bounds__(256) k_step_pair(const RepDev* __restrict__ reps,
                                                   const BlockEntry* __restrict__ blocks,
                                                   const PairTable<T> tab, int32_t flags,
                                                   double* __restrict__ partials, int n_rep,
                                                   int32_t* __restrict__ status,
                                                   const StepRef sync, int W,
                                                   const T* __restrict__ zeta_row)
{
    using V4 = typename NV<T>::v4;
    using T4 = typename Vec4<T>::type;
    constexpr int NCH = 64 / G;
    __shared__ double part[4][G][5];
    __shared__ double red[4][kNobs];
    __shared__ double tx[256], ty[256], tz[256], td[256];
    __shared__ double dmax_s[4];
    // the update's inputs, staged before the force loop: C, the ring
    // propagators, and per (atom slot, component, bead / mode) positions,
    // velocities and noise
    __shared__ double Cs[G * G], ringS[3 * G];
    __shared__ double xs[4][3][G], vs[4][3][G], zsh[4][3][G];
    const StepIdx si = step_index(sync);
    const int pin = si.p, pout = si.p ^ 1;
    const int fnext = si.f == 2 ? 0 : si.f + 1, fold = si.f == 0 ? 2 : si.f - 1;
    if (blockIdx.x == 0) {  // flags of step n - 1 are not read again until step n + 2
        for (int r = threadIdx.x; r < n_rep; r += blockDim.x) reps[r].rflag[fold] = 0;
        if (threadIdx.x == 0) status[kAnyRebuild + fold] = 0;
    }
    const int lb = xcd_block();
    const BlockEntry be = blocks[lb];
    const int rep = __builtin_amdgcn_readfirstlane(be.rep);
    const RepDev& R = reps[rep];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = wave / W, wsub = wave % W;
    const int bl = lane % G, ch = lane / G + wsub * NCH;
    const int i = be.atom0 + slot;
    const int N = R.N, P = R.P;
    const bool active = i < N;
    const int s = bl;  // G = P: the wavefront holds every bead
    constexpr bool want_e = WE;  // = flags & kSample (the launcher's choice)
    double* const vrec = recorder_row(R, flags);
    __shared__ f4v ltab[2 * kPairs];
    fill_ltab<T, NS, FAST>(tab, ltab);
    {
        const int apb = 4 / W;
        for (int t = threadIdx.x; t < G * G; t += blockDim.x) Cs[t] = R.nm[t];
        for (int t = threadIdx.x; t < 3 * G; t += blockDim.x) ringS[t] = R.ring[t];
        for (int t = threadIdx.x; t < apb * 3 * G; t += blockDim.x) {
            const int sl = t / (3 * G), rem = t % (3 * G), a = rem / G, b = rem % G;
            const int ii = be.atom0 + sl;
            if (ii < N) {
                const size_t idx = ((size_t)b * 3 + a) * N + ii;
                xs[sl][a][b] = R.pos[idx];
                vs[sl][a][b] = R.vel[idx];
                zsh[sl][a][b] = (double)zeta_row[R.dof_off + ((int64_t)3 * ii + a) * P + b];
            }
        }
    }
    __syncthreads();
    const bool rebuild = R.rflag[si.f] != 0;  // uniform over the block
    const double* __restrict__ cin = R.cnb[pin];
    const double* __restrict__ rin = R.rrefb[pin];
    if (rebuild)
        rebuild_list<T>(R, i, active && wsub == 0, cin, cin + N, cin + 2 * (size_t)N, R.devn[pin],
                        status, tx, ty, tz, td, dmax_s, 1.0);
    double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0, vir = 0.0;
    int spi = 0;
    if (active) {
        if (rebuild) {
            const PairPos<T, kPosRecon> pp{(gptr<V4>)R.ub[pin] + 0, (gptr<double>)rin,
                                           (gptr<double>)cin, N, P, nullptr, nullptr};
            pair_sum<T, NS, FAST, DEG, kPosRecon, G>(R, tab, pp, i, s, ch, NCH * W, want_e, want_e,
                                                  fx, fy, fz, e, vir, spi, 1.0, ltab);
        } else {
            // (no barostat with the one-kernel step)
            const PairPos<T, kPosDirect> pp{(gptr<V4>)R.ub[pin] + 0, nullptr, nullptr, N, P,
                                            nullptr, nullptr};
            pair_sum<T, NS, FAST, DEG, kPosDirect, G>(R, tab, pp, i, s, ch, NCH * W, want_e,
                                                   want_e, fx, fy, fz, e, vir, spi, R.npt_S, ltab);
        }
    }
    reduce_atom<G>(fx, fy, fz, e, vir, want_e, want_e, W, wave, wsub, lane, part);
    double ob[kNobs] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int my_flags = 0;
    // the atom's wavefront, lanes 0 .. P-1 = beads: wavefront-uniform branch.
    if (active && wsub == 0) {
        const bool own = lane < G;
        struct LdsState {
            const double (*x)[G];
            const double (*v)[G];
            __device__ __forceinline__ double pos(int b, int a) const { return x[a][b]; }
            __device__ __forceinline__ double vel(int b, int a) const { return v[a][b]; }
        };
        const LdsState src{xs[slot], vs[slot]};
        double vc[3] = {0.0, 0.0, 0.0};   // velocities after the closing half-kick
        double fT[3] = {0.0, 0.0, 0.0};
        if (own) {
            const double f[3] = {fx, fy, fz};
            force_epilogue_src<T, false>(R, i, s, spi, f, 0.5 * e, kKick | (flags & kSample), ob,
                                         src, vc, vrec);
            if (flags & kSample) ob[5] = 0.5 * vir;
#pragma unroll
            for (int a = 0; a < 3; ++a) fT[a] = (double)(T)f[a];  // the stored force
        }
        if (flags & kSample) {
            // kinetic energy of the centroid, (1/2) m |sum_s v_s|^2 / P: the
            // wavefront holds every bead (G = P), lanes >= G hold zeros
            double ck = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                double vs = 0.0;
#pragma unroll
                for (int b = 0; b < G; ++b) vs += __shfl(vc[a], b);
                ck = __builtin_fma(vs, vs, ck);
            }
            if (lane == 0) ob[6] = 0.5 * R.mmu[spi] * ck / P;
        }
        const int k = s;  // after the transform this lane holds mode k
        double cw = 0.0, sw = 0.0, ws = 0.0, kick = 0.0, sig = 0.0;
        if (own) {
            cw = ringS[k];
            sw = ringS[P + k];
            ws = ringS[2 * P + k];
            kick = R.kick[spi];
            sig = R.sigma[spi];
        }
        double rn[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const size_t idx = ((size_t)s * 3 + a) * N + i;
            double r = 0.0, v = 0.0;
            if (own) {
                r = xs[slot][a][s];
                v = half_kick(vc[a], kick, fT[a]);  // opening half-kick of step n
            }
            double q = 0.0, pm = 0.0;
#pragma unroll
            for (int b = 0; b < G; ++b) {
                const double c = own ? Cs[b * P + k] : 0.0;
                q = nm_acc(q, c, xs[slot][a][b]);
                pm = nm_acc(pm, c, __shfl(v, b));
            }
            if (own) mode_aoa(q, pm, cw, sw, ws, R.c1, sig, zsh[slot][a][k]);
            double x = 0.0, y = 0.0;
#pragma unroll
            for (int kk = 0; kk < G; ++kk) {
                const double c = own ? Cs[s * P + kk] : 0.0;
                x = nm_acc(x, c, __shfl(q, kk));
                y = nm_acc(y, c, __shfl(pm, kk));
            }
            if (own) {
                R.pos[idx] = x;
                R.vel[idx] = y;
                if (!(__builtin_isfinite(x) && __builtin_isfinite(y))) my_flags |= kStatusNonfinite;
            }
            rn[a] = x;
        }
        // centroid (bead order), new references, relative positions, spread
        double cen[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
        for (int b = 0; b < G; ++b) {
#pragma unroll
            for (int a = 0; a < 3; ++a) cen[a] += __shfl(rn[a], b);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) cen[a] /= P;
        if (own) {
            double ref[3], devb;
            if (rebuild) {
#pragma unroll
                for (int a = 0; a < 3; ++a) ref[a] = cin[(size_t)a * N + i];
                devb = R.devn[pin][i];
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a) ref[a] = rin[(size_t)a * N + i];
                devb = R.devbb[pin][i];
            }
            double u3[3], u2 = 0.0, d2 = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                u3[a] = rn[a] - ref[a];
                u2 = nm_acc(u2, u3[a], u3[a]);
                const double dc = rn[a] - cen[a];
                d2 = nm_acc(d2, dc, dc);
            }
            T4 val;
            val.x = (T)u3[0];
            val.y = (T)u3[1];
            val.z = (T)u3[2];
            val.w = as_bits_t<T>(spi);
            ((T4*)R.ub[pout])[(size_t)i * P + s] = val;
            const double lim = devb + R.half_skin;
            if (!(u2 <= lim * lim)) my_flags |= 8;
            double dm = d2;
            for (int b = 0; b < G; ++b) dm = fmax(dm, __shfl(d2, b));
            if (lane == 0) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    R.cnb[pout][(size_t)a * N + i] = cen[a];
                    R.rrefb[pout][(size_t)a * N + i] = ref[a];
                }
                R.devn[pout][i] = sqrt(dm);
                R.devbb[pout][i] = devb;
            }
        }
    }
    // flags of the step: one atomic per wavefront
    for (int off = 1; off < 64; off <<= 1) my_flags |= __shfl_xor(my_flags, off);
    if (lane == 0 && my_flags) {
        if (my_flags & 8) {
            atomicOr(R.rflag + fnext, 1);
            atomicOr(status + kAnyRebuild + fnext, 1);
        }
        if (my_flags & kStatusNonfinite) atomicOr(status, kStatusNonfinite);
    }
    if (flags & kSample) block_partials(ob, wave, lane, lb, red, partials);
}

// On-site potential of one dof, V(x) and F = -dV/dx (FP64): harmonic with
// k = m omega_i^2, Morse V0 (1 - e^{-x/d})^2, double well V0 ((x/d)^2 - 1)^2.
template <int KIND>
__device__ __forceinline__ double onsite(double x, double k, double V0, double d, double& F)
{
    if constexpr (KIND == QTB_POT_HARMONIC) {
        F = -k * x;
        return 0.5 * k * x * x;
    } else if constexpr (KIND == QTB_POT_MORSE) {
        const double e = exp(-x / d);
        F = -2.0 * V0 * (1.0 - e) * e / d;
        return V0 * (1.0 - e) * (1.0 - e);
    } else {
        const double y = x / d, w = y * y - 1.0;
        F = -4.0 * V0 * w * y / d;
        return V0 * w * w;
    }
}

// Independent oscillators (every dof alone): V = sum over dofs of the
// on-site potential per bead.
template <typename T, int KIND>
__global__ void __launch_bounds__(256) k_force_onsite(const RepDev* __restrict__ reps,
                                                      const BlockEntry* __restrict__ blocks,
                                                      int32_t flags, double* __restrict__ partials)
{
    __shared__ double red[4][kNobs];
    const BlockEntry be = blocks[blockIdx.x];
    const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
    const int i = be.atom0 + threadIdx.x;
    const int N = R.N, P = R.P, dims = R.dims;
    double ob[kNobs] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < N) {
        const int sp = R.species[i];
        const double m = R.mmu[sp], kick = R.kick[sp];
        const double k = KIND == QTB_POT_HARMONIC ? m * R.homega[i] * R.homega[i] : 0.0;
        const double V0 = R.osV0[sp], dl = R.osd[sp];
        double* vrow = recorder_row(R, flags);  // velocity recorder (P = 1)
        if (vrow) vrow += i;
        double ke = 0.0, U = 0.0, spr = 0.0, vir = 0.0, x2 = 0.0;
        for (int a = 0; a < dims; ++a) {
            double c = 0.0;
            for (int s = 0; s < P; ++s) c += R.pos[((size_t)s * dims + a) * N + i];
            c /= P;
            for (int s = 0; s < P; ++s) {
                const size_t idx = ((size_t)s * dims + a) * N + i;
                const double x = R.pos[idx];
                double f;
                const double Vx = onsite<KIND>(x, k, V0, dl, f);
                ((T*)R.force)[idx] = (T)f;
                double v = R.vel[idx];
                if (flags & kKick) {
                    v += kick * f;
                    R.vel[idx] = v;
                }
                if (vrow) vrow[(size_t)a * N] = v;
                if (flags & (kSample | kEvaluate)) {
                    const int sn = (s + 1 == P) ? 0 : s + 1;
                    const double dn = x - R.pos[((size_t)sn * dims + a) * N + i];
                    const double d0 = x - R.r0[idx];
                    ke += 0.5 * m * v * v;
                    U += Vx;
                    spr += dn * dn;
                    vir += (x - c) * f;
                    x2 += d0 * d0;
                    if (flags & kEvaluate) {
                        double* ea = R.eatom + (size_t)s * N + i;
                        *ea = (a == 0 ? 0.0 : *ea) + Vx;
                    }
                }
            }
        }
        ob[0] = ke;
        ob[1] = U / P;
        ob[2] = (P > 1) ? 0.5 * m * R.omega_P * R.omega_P * spr : 0.0;
        ob[3] = vir;
        ob[4] = x2;
    }
    if (flags & kSample) {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
        for (int q = 0; q < kNobs; ++q) {
            const double t = wave_sum(ob[q]);
            if (lane == 0) red[wave][q] = t;
        }
        __syncthreads();
        if (threadIdx.x < kNobs) {
            const double t = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                             red[3][threadIdx.x];
            partials[(size_t)blockIdx.x * kNobs + threadIdx.x] = t;
        }
    }
}

// Kinetic energy of the ring-polymer centroids (normal mode k = 0),
// sum_i (1/2) m_i |sum_s v_i^(s)|^2 / P = sum_i (1/2) m_i P |v_c,i|^2, of
// replica blockIdx.y in chunks of kCentroidChunk atoms (chunk blockIdx.x);
// fixed-order sums, one value per chunk into cpart[rep][cchunks].
__global__ void __launch_bounds__(kCentroidChunk) k_centroid_ke(const RepDev* __restrict__ reps,
                                                                double* __restrict__ cpart,
                                                                int cchunks)
{
    __shared__ double red[kCentroidChunk / 64];
    const int r = blockIdx.y;
    const RepDev& R = reps[r];
    const int i0 = blockIdx.x * kCentroidChunk;
    if (i0 >= R.N) return;  // uniform: chunks past the replica's atoms stay unread
    const int i = i0 + threadIdx.x;
    double k = 0.0;
    if (i < R.N) {
        const int N = R.N, P = R.P, dims = R.dims;
        for (int a = 0; a < dims; ++a) {
            double vs = 0.0;
            for (int b = 0; b < P; ++b) vs += R.vel[((size_t)b * dims + a) * N + i];
            k = __builtin_fma(vs, vs, k);
        }
        k *= 0.5 * R.mmu[R.species[i]] / P;
    }
    k = wave_sum(k);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wave] = k;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kCentroidChunk / 64; ++w) t += red[w];
        cpart[(size_t)r * cchunks + blockIdx.x] = t;
    }
}

// Per replica (one workgroup each): acc += sum of the replica's block
// partials.  Thread t sums blocks t, t + 256, ... in order, then a fixed
// tree in LDS: the same order on every run and for a replica alone or in a
// batch (the assignment is relative to the replica's first block).
__global__ void __launch_bounds__(256) k_obs_reduce(const RepDev* __restrict__ reps, int n_rep,
                                                    const double* __restrict__ partials,
                                                    double* __restrict__ acc,
                                                    int32_t* __restrict__ counts, int tick,
                                                    int pair, const double* __restrict__ cpart,
                                                    int cchunks)
{
    __shared__ double red[kNobs][256];
    const int r = blockIdx.x;
    if (r >= n_rep) return;
    const RepDev& R = reps[r];
    double t[kNobs] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < R.obs_nblocks; b += blockDim.x)
        for (int q = 0; q < kNobs; ++q) t[q] += partials[(size_t)(R.obs_block0 + b) * kNobs + q];
    for (int q = 0; q < kNobs; ++q) red[q][threadIdx.x] = t[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int q = 0; q < kNobs; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    double* a = acc + (size_t)r * kAcc;
    if (threadIdx.x < kNobs) a[threadIdx.x] += red[threadIdx.x][0];
    if (threadIdx.x == 0) {
        counts[r] += 1;
        if (tick && R.vt) *R.vt_n += 1;  // the forces of this sample wrote its row
        if (cpart) {  // centroid kinetic energy, chunks in order
            double kc = 0.0;
            const int nc = (R.N + kCentroidChunk - 1) / kCentroidChunk;
            for (int q = 0; q < nc; ++q) kc += cpart[(size_t)r * cchunks + q];
            a[6] += kc;
        }
        if (pair) {
            // volume of this sample's box (it changes under the barostat: the
            // positions already carry the pending factor npt_sr, the box
            // takes it at the end of the step) and the primitive pressure
            // (2K - 2 U_spring + W / P) / (3V)
            const double sr = R.npt_sr;
            const double V = (R.box[0] * sr) * (R.box[1] * sr) * (R.box[2] * sr);
            a[kNobs] += V;
            a[kNobs + 1] += (2.0 * red[0][0] - 2.0 * red[2][0] + red[5][0] / R.P) / (3.0 * V);
        }
    }
}

__global__ void k_fill(int32_t* __restrict__ p, int64_t n, int32_t v)
{
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n;
         id += (int64_t)gridDim.x * blockDim.x)
        p[id] = v;
}

template <typename T, int NS, bool FAST, int DEG, int EM>
void launch_pair_GW(hipStream_t st, int G, const RepDev* reps, const BlockEntry* blocks,
                    int n_blocks, const PairTable<T>& tab, int32_t flags, double* partials,
                    int clear, int n_rep, int32_t* status, StepRef sync, int W)
{
    const dim3 g(n_blocks), b(256);
    switch (G) {
    case 1: launch((k_force_pair<T, 1, NS, FAST, DEG, EM>), g, b, 0, st, reps, blocks, tab, flags, partials, clear, n_rep, status, sync, W); break;
    case 2: launch((k_force_pair<T, 2, NS, FAST, DEG, EM>), g, b, 0, st, reps, blocks, tab, flags, partials, clear, n_rep, status, sync, W); break;
    case 4: launch((k_force_pair<T, 4, NS, FAST, DEG, EM>), g, b, 0, st, reps, blocks, tab, flags, partials, clear, n_rep, status, sync, W); break;
    case 8: launch((k_force_pair<T, 8, NS, FAST, DEG, EM>), g, b, 0, st, reps, blocks, tab, flags, partials, clear, n_rep, status, sync, W); break;
    default: break;
    }
}
template <typename T, int NS, bool FAST, int DEG>
void launch_pair_G(hipStream_t st, int G, const RepDev* reps, const BlockEntry* blocks,
                   int n_blocks, const PairTable<T>& tab, int32_t flags, double* partials,
                   int clear, int n_rep, int32_t* status, StepRef sync, int W)
{
    if (flags & (kSample | kEvaluate))
        launch_pair_GW<T, NS, FAST, DEG, 2>(st, G, reps, blocks, n_blocks, tab, flags, partials,
                                            clear, n_rep, status, sync, W);
    else if (flags & kPressure)
        launch_pair_GW<T, NS, FAST, DEG, 1>(st, G, reps, blocks, n_blocks, tab, flags, partials,
                                            clear, n_rep, status, sync, W);
    else
        launch_pair_GW<T, NS, FAST, DEG, 0>(st, G, reps, blocks, n_blocks, tab, flags, partials,
                                            clear, n_rep, status, sync, W);
}

template <typename T, bool FAST, int DEG>
void launch_pair_T(hipStream_t st, int G, const RepDev* reps, const BlockEntry* blocks,
                   int n_blocks, const PairTable<T>& tab, int32_t flags, double* partials,
                   int clear, int n_rep, int32_t* status, StepRef sync, int W)
{
    if (tab.n_species <= 2)
        launch_pair_G<T, 2, FAST, DEG>(st, G, reps, blocks, n_blocks, tab, flags, partials, clear, n_rep, status, sync, W);
    else
        launch_pair_G<T, 4, FAST, DEG>(st, G, reps, blocks, n_blocks, tab, flags, partials, clear, n_rep, status, sync, W);
}

}  // namespace

void launch_forces_pair(hipStream_t st, bool fp64, int G, int W, const RepDev* reps,
                        const BlockEntry* blocks, int n_blocks, const void* table, int32_t flags,
                        double* partials, int clear, int n_rep, int32_t* status,
                        StepRef sync)
{
    if (fp64) {
        launch_pair_T<double, false, 1>(st, G, reps, blocks, n_blocks,
                                     *(const PairTable<double>*)table, flags, partials,
                                     clear, n_rep, status, sync, W);
    } else {
        const PairTable<float>& t = *(const PairTable<float>*)table;
        if (t.ex_deg == 10)
            launch_pair_T<float, true, 10>(st, G, reps, blocks, n_blocks, t, flags, partials,
                                           clear, n_rep, status, sync, W);
        else if (t.ex_deg == kErfcxMaxDeg)
            launch_pair_T<float, true, kErfcxMaxDeg>(st, G, reps, blocks, n_blocks, t, flags,
                                                     partials, clear, n_rep, status, sync, W);
        else
            launch_pair_T<float, false, 1>(st, G, reps, blocks, n_blocks, t, flags, partials,
                                           clear, n_rep, status, sync, W);
    }
}

template <typename T, int NS, bool FAST, int DEG, bool WE>
void launch_step_GW(hipStream_t st, int G, const RepDev* reps, const BlockEntry* blocks,
                    int n_blocks, const PairTable<T>& tab, int32_t flags, double* partials,
                    int n_rep, int32_t* status, StepRef sync, int W, const T* zrow)
{
    const dim3 g(n_blocks), b(256);
    switch (G) {
    case 1: launch((k_step_pair<T, 1, NS, FAST, DEG, WE>), g, b, 0, st, reps, blocks, tab, flags, partials, n_rep, status, sync, W, zrow); break;
    case 2: launch((k_step_pair<T, 2, NS, FAST, DEG, WE>), g, b, 0, st, reps, blocks, tab, flags, partials, n_rep, status, sync, W, zrow); break;
    case 4: launch((k_step_pair<T, 4, NS, FAST, DEG, WE>), g, b, 0, st, reps, blocks, tab, flags, partials, n_rep, status, sync, W, zrow); break;
    case 8: launch((k_step_pair<T, 8, NS, FAST, DEG, WE>), g, b, 0, st, reps, blocks, tab, flags, partials, n_rep, status, sync, W, zrow); break;
    default: break;
    }
}
template <typename T, int NS, bool FAST, int DEG>
void launch_step_G(hipStream_t st, int G, const RepDev* reps, const BlockEntry* blocks,
                   int n_blocks, const PairTable<T>& tab, int32_t flags, double* partials,
                   int n_rep, int32_t* status, StepRef sync, int W, const T* zrow)
{
    if (flags & kSample)
        launch_step_GW<T, NS, FAST, DEG, true>(st, G, reps, blocks, n_blocks, tab, flags, partials,
                                               n_rep, status, sync, W, zrow);
    else
        launch_step_GW<T, NS, FAST, DEG, false>(st, G, reps, blocks, n_blocks, tab, flags, partials,
                                                n_rep, status, sync, W, zrow);
}

template <typename T, bool FAST, int DEG>
void launch_step_T(hipStream_t st, int G, const RepDev* reps, const BlockEntry* blocks,
                   int n_blocks, const PairTable<T>& tab, int32_t flags, double* partials,
                   int n_rep, int32_t* status, StepRef sync, int W, const T* zrow)
{
    if (tab.n_species <= 2)
        launch_step_G<T, 2, FAST, DEG>(st, G, reps, blocks, n_blocks, tab, flags, partials, n_rep, status, sync, W, zrow);
    else
        launch_step_G<T, 4, FAST, DEG>(st, G, reps, blocks, n_blocks, tab, flags, partials, n_rep, status, sync, W, zrow);
}

void launch_step_pair(hipStream_t st, bool fp64, int G, int W, const RepDev* reps,
                      const BlockEntry* blocks, int n_blocks, const void* table, int32_t flags,
                      double* partials, int n_rep, int32_t* status, StepRef sync,
                      const void* zeta_row)
{
    if (fp64) {
        launch_step_T<double, false, 1>(st, G, reps, blocks, n_blocks,
                                        *(const PairTable<double>*)table, flags, partials, n_rep,
                                        status, sync, W, (const double*)zeta_row);
    } else {
        const PairTable<float>& t = *(const PairTable<float>*)table;
        const float* z = (const float*)zeta_row;
        if (t.ex_deg == 10)
            launch_step_T<float, true, 10>(st, G, reps, blocks, n_blocks, t, flags, partials, n_rep, status, sync, W, z);
        else if (t.ex_deg == kErfcxMaxDeg)
            launch_step_T<float, true, kErfcxMaxDeg>(st, G, reps, blocks, n_blocks, t, flags, partials, n_rep, status, sync, W, z);
        else
            launch_step_T<float, false, 1>(st, G, reps, blocks, n_blocks, t, flags, partials, n_rep, status, sync, W, z);
    }
}

void launch_forces_onsite(hipStream_t st, bool fp64, int kind, const RepDev* reps,
                          const BlockEntry* blocks, int n_blocks, int32_t flags,
                          double* partials)
{
    const dim3 g(n_blocks), b(256);
    if (fp64) {
        if (kind == QTB_POT_MORSE)
            launch((k_force_onsite<double, QTB_POT_MORSE>), g, b, 0, st, reps, blocks, flags, partials);
        else if (kind == QTB_POT_DOUBLE_WELL)
            launch((k_force_onsite<double, QTB_POT_DOUBLE_WELL>), g, b, 0, st, reps, blocks, flags,
                   partials);
        else
            launch((k_force_onsite<double, QTB_POT_HARMONIC>), g, b, 0, st, reps, blocks, flags,
                   partials);
    } else {
        if (kind == QTB_POT_MORSE)
            launch((k_force_onsite<float, QTB_POT_MORSE>), g, b, 0, st, reps, blocks, flags, partials);
        else if (kind == QTB_POT_DOUBLE_WELL)
            launch((k_force_onsite<float, QTB_POT_DOUBLE_WELL>), g, b, 0, st, reps, blocks, flags,
                   partials);
        else
            launch((k_force_onsite<float, QTB_POT_HARMONIC>), g, b, 0, st, reps, blocks, flags,
                   partials);
    }
}

void launch_obs_reduce(hipStream_t st, const RepDev* reps, int n_rep, const double* partials,
                       double* acc, int32_t* counts, bool tick, bool pair, double* cpart,
                       int cchunks)
{
    if (cpart)
        launch(k_centroid_ke, dim3(cchunks, n_rep), dim3(kCentroidChunk), 0, st, reps, cpart,
               cchunks);
    launch(k_obs_reduce, dim3(n_rep), dim3(256), 0, st, reps, n_rep, partials, acc, counts,
           tick ? 1 : 0, pair ? 1 : 0, (const double*)cpart, cchunks);
}

void launch_fill(hipStream_t st, void* p, int64_t n_words, int32_t value)
{
    if (n_words <= 0) return;
    int64_t blocks = (n_words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    launch(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, (int32_t*)p, n_words,
                       value);
}

}  // namespace qtb
