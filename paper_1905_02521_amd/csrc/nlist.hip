// nlist.hip -- Verlet neighbour lists shared by all beads of a replica.
//
// The list is built from the bead centroids r_ref with radius r_cut + skin
// and stores, per entry, the reference displacement d_ij = r_ref_i - r_ref_j
// - S (S the periodic image shift) plus j.  Every bead then measures a pair
// as d_ij + u_i - u_j with u = r - r_ref small, which keeps the FP32 force
// path accurate at any box size and lets positions stay unwrapped.  All
// periodic images within range are listed (boxes smaller than twice the
// cut-off, e.g. 3x3x3 rock-salt cells at r_cut = 9 A, need them).
//
// Both kernels run every step and return at once unless the update kernel
// flagged that some bead moved more than skin / (2 sqrt 3) per component
// from its reference (then no pair within r_cut can be missing from the
// list).  The build is all-pairs with j tiles staged in LDS: deterministic
// order (j ascending, images in a fixed order), rebuilt rarely.
#include "qtb_internal.h"

namespace qtb {
namespace {

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

__device__ __forceinline__ float bits_f(int32_t b, float) { return __int_as_float(b); }
__device__ __forceinline__ double bits_f(int32_t b, double) { return __longlong_as_double((long long)b); }

// New references (bead centroids) and positions relative to them.
template <typename T>
__global__ void __launch_bounds__(256) k_nlist_refs(const RepDev* __restrict__ reps,
                                                    const BlockEntry* __restrict__ blocks)
{
    using T4 = typename Vec4<T>::type;
    const BlockEntry be = blocks[blockIdx.x];
    const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
    if (*R.rebuild == 0) return;
    const int i = be.atom0 + threadIdx.x;
    const int N = R.N, P = R.P;
    if (i >= N) return;
    double c[3];
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int b = 0; b < P; ++b) s += R.pos[((size_t)b * 3 + a) * N + i];
        c[a] = s / P;
        R.rref[(size_t)a * N + i] = c[a];
    }
    T4* __restrict__ u = (T4*)R.u;
    const T spb = bits_f(R.species[i], T());
    for (int b = 0; b < P; ++b) {
        T4 v;
        v.x = (T)(R.pos[((size_t)b * 3 + 0) * N + i] - c[0]);
        v.y = (T)(R.pos[((size_t)b * 3 + 1) * N + i] - c[1]);
        v.z = (T)(R.pos[((size_t)b * 3 + 2) * N + i] - c[2]);
        v.w = spb;
        u[(size_t)b * N + i] = v;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_nlist_build(const RepDev* __restrict__ reps,
                                                     const BlockEntry* __restrict__ blocks,
                                                     int32_t* __restrict__ status)
{
    using T4 = typename Vec4<T>::type;
    __shared__ double sx[256], sy[256], sz[256];
    const BlockEntry be = blocks[blockIdx.x];
    const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
    if (*R.rebuild == 0) return;  // uniform over the block
    const int N = R.N;
    const int i = be.atom0 + threadIdx.x;
    const bool active = i < N;
    const double Lx = R.box[0], Ly = R.box[1], Lz = R.box[2];
    const double R2 = R.r_skin2;
    const double Rl = sqrt(R2);
    const int mx = (int)ceil(Rl / Lx - 0.5), my = (int)ceil(Rl / Ly - 0.5),
              mz = (int)ceil(Rl / Lz - 0.5);
    double xi = 0.0, yi = 0.0, zi = 0.0;
    if (active) {
        xi = R.rref[i];
        yi = R.rref[(size_t)N + i];
        zi = R.rref[(size_t)2 * N + i];
    }
    T4* __restrict__ ent = (T4*)R.nb_entries + (size_t)i * R.maxnb;
    int cnt = 0;
    for (int j0 = 0; j0 < N; j0 += 256) {
        __syncthreads();
        const int jl = j0 + threadIdx.x;
        if (jl < N) {
            sx[threadIdx.x] = R.rref[jl];
            sy[threadIdx.x] = R.rref[(size_t)N + jl];
            sz[threadIdx.x] = R.rref[(size_t)2 * N + jl];
        }
        __syncthreads();
        if (!active) continue;
        const int jn = min(256, N - j0);
        for (int jj = 0; jj < jn; ++jj) {
            const int j = j0 + jj;
            double dx = xi - sx[jj], dy = yi - sy[jj], dz = zi - sz[jj];
            dx -= Lx * rint(dx / Lx);
            dy -= Ly * rint(dy / Ly);
            dz -= Lz * rint(dz / Lz);
            for (int nx = -mx; nx <= mx; ++nx) {
                const double ex = dx + nx * Lx;
                const double ex2 = ex * ex;
                if (ex2 >= R2) continue;
                for (int ny = -my; ny <= my; ++ny) {
                    const double ey = dy + ny * Ly;
                    const double exy2 = ex2 + ey * ey;
                    if (exy2 >= R2) continue;
                    for (int nz = -mz; nz <= mz; ++nz) {
                        const double ez = dz + nz * Lz;
                        const double r2 = exy2 + ez * ez;
                        if (r2 >= R2) continue;
                        if (j == i && nx == 0 && ny == 0 && nz == 0) continue;
                        if (cnt < R.maxnb) {
                            T4 v;
                            v.x = (T)ex;
                            v.y = (T)ey;
                            v.z = (T)ez;
                            v.w = bits_f(j, T());
                            ent[cnt] = v;
                        }
                        ++cnt;
                    }
                }
            }
        }
    }
    if (active) {
        R.nb_count[i] = min(cnt, R.maxnb);
        if (cnt > R.maxnb) atomicOr(status, kStatusNbOverflow);
    }
}

}  // namespace

void launch_nlist(hipStream_t st, bool fp64, const RepDev* reps, const BlockEntry* blocks,
                  int n_blocks, int32_t* status)
{
    if (fp64) {
        hipLaunchKernelGGL(k_nlist_refs<double>, dim3(n_blocks), dim3(256), 0, st, reps, blocks);
        hipLaunchKernelGGL(k_nlist_build<double>, dim3(n_blocks), dim3(256), 0, st, reps, blocks,
                           status);
    } else {
        hipLaunchKernelGGL(k_nlist_refs<float>, dim3(n_blocks), dim3(256), 0, st, reps, blocks);
        hipLaunchKernelGGL(k_nlist_build<float>, dim3(n_blocks), dim3(256), 0, st, reps, blocks,
                           status);
    }
}

}  // namespace qtb
