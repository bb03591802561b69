// pairsym.hpp -- the all-pairs ion-ion sum with each pair evaluated once.
//
// The screened Coulomb force is antisymmetric, so the tile pair (I, J) of
// 256-ion target and source tiles also gives the reaction on the sources.
// Work items are runs of tiles J in [J0, J1) of kSymRows consecutive target
// tile rows I .. I + kSymRows - 1 (J >= I), longest first; small systems take
// one target row per item.  Within an item:
//   * the rows' own tiles (J < I + kSymRows) go one row at a time, with the
//     diagonal tile (J == I) summed one-sided (each ordered pair);
//   * an off-diagonal tile is cut into four sub-tiles of 64 sources; lane l of
//     a wave holds one target of every row of the item and meets source
//     (l + k) mod 64 in step k, adds each term to that target's sum and
//     subtracts it from a source accumulator that moves one lane down each
//     step (a wavefront rotate), so that after 64 steps every lane holds the
//     reaction on one source, summed over the wave's targets in a fixed
//     order; the four waves' sums are added in LDS in a fixed order;
//   * reactions go to the sources' int64 fixed-point accumulators once per
//     tile, and the targets' sums once per item.
// Fixed-point integer addition is exact and commutative, so the totals do
// not depend on the order in which items run: results are deterministic.
// The step's tail kernel converts the totals, adds the grain, drive and
// confinement terms and the Eq. (1) sums, and clears the accumulators for
// the next step.
#pragma once

#include "kernels.hpp"
#include "symitems.hpp"

namespace odk {

// The accumulators hold the raw sums (1 + r) e^-r / r^3 d times a per-system
// power of two, PairArgs::sym_scale, set by the host from the ion density so
// that the resolution stays near 1e-8 of a typical sum (dominated by the
// nearest neighbours, ~ n^(2/3)) while the int64 range keeps a margin of
// about 1e13 for close pairs.

// The occupancy the symmetric kernels are compiled for, with kSymRows = 3
// target rows per item (symitems.hpp).  Three rows at six waves per SIMD,
// with the step written as differences, pair terms, then sums and all 64
// steps of a sub-tile unrolled, timed fastest among 2 to 4 rows, four
// statement orders, 16, 32 or 64 unrolled steps and 5 to 8 waves per SIMD
// on gfx950.
constexpr int kSymWaves = 6;

// One pair term (1 + r) e^-r / r^3 for the difference d, as E / r + E with
// E = e^-r / r^2 = 2^-(r log2(e) + log2(r^2)): the 1/r^2 factor rides in the
// exponent, so the term takes six ordinary instructions and three
// transcendental ones (rsq, log2, exp2), which the SIMD largely overlaps with
// the ordinary instructions of the other rows.  A sentinel far away
// (r ~ 1e18) gives E = 0 exactly.
__device__ __forceinline__ float sym_f(float dx, float dy, float dz)
{
    const float kNegLog2e = -1.4426950408889634f;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ri;
    const float E = __builtin_amdgcn_exp2f(fmaf(r, kNegLog2e, -__builtin_amdgcn_logf(r2)));
    return fmaf(E, ri, E);
}

// The screened Coulomb pair term as a functor for sym_item.
struct PlainPair {
    __device__ __forceinline__ float operator()(float dx, float dy, float dz) const { return sym_f(dx, dy, dz); }
};

__device__ __forceinline__ float rotate_down(float v)
{
    // lane l receives the value of lane l + 1 (mod 64): DPP wave_rol:1
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x134, 0xf,
                                                              0xf, true));
}

// One work item of one system (positions X, Y, Z; N ions): target tile row
// I against the 64-ion sub-tiles [st0, st1) of the source tiles [J0, J1),
// J0 >= I.  Reactions go to fix[c * stride + j], the targets' sums to
// fix[c * stride + i] (indices local to the system).  pair(d) is the scalar
// f of the term f d.
template <int BLOCK, typename Pair>
__device__ __forceinline__ void sym_item(const float* __restrict__ X, const float* __restrict__ Y,
                                         const float* __restrict__ Z, int N, int I, int J0, int J1,
                                         int st0, int st1, unsigned long long* __restrict__ fix,
                                         long long stride, double scale, int* status, float4 (*src)[128],
                                         float (*jpart)[3][BLOCK], const Pair& pair)
{
    static_assert(BLOCK == 256, "four waves of 64");
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = I * BLOCK + threadIdx.x;
    const float xi = X[i], yi = Y[i], zi = Z[i];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int J = J0; J < J1; ++J) {
        const int j0 = J * BLOCK;
        __syncthreads();
        {
            const int st = threadIdx.x >> 6, l = threadIdx.x & 63;
            const float4 q = make_float4(X[j0 + threadIdx.x], Y[j0 + threadIdx.x], Z[j0 + threadIdx.x], 0.0f);
            src[st][l] = q;
            src[st][l + 64] = q;
        }
        __syncthreads();
        float ax = 0.0f, ay = 0.0f, az = 0.0f;
        if (J == I) {
            for (int k = 64 * st0; k < 64 * st1; ++k) {
                const float4 q = src[k >> 6][k & 63];
                const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
                float f = pair(dx, dy, dz);
                f = (k == (int)threadIdx.x) ? 0.0f : f;
                ax = fmaf(f, dx, ax);
                ay = fmaf(f, dy, ay);
                az = fmaf(f, dz, az);
            }
        } else {
            for (int st = st0; st < st1; ++st) {
                float jx = 0.0f, jy = 0.0f, jz = 0.0f;
                const float4* base = &src[st][lane];
#pragma unroll 16
                for (int k = 0; k < 64; ++k) {
                    const float4 q = base[k];                 // source (lane + k) mod 64
                    const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
                    const float f = pair(dx, dy, dz);
                    ax = fmaf(f, dx, ax);
                    ay = fmaf(f, dy, ay);
                    az = fmaf(f, dz, az);
                    jx = fmaf(-f, dx, rotate_down(jx));
                    jy = fmaf(-f, dy, rotate_down(jy));
                    jz = fmaf(-f, dz, rotate_down(jz));
                }
                // after 64 rotations lane l holds source (l + 63) mod 64
                const int sid = st * 64 + ((lane + 63) & 63);
                jpart[wv][0][sid] = jx;
                jpart[wv][1][sid] = jy;
                jpart[wv][2][sid] = jz;
            }
            __syncthreads();
            const int j = j0 + threadIdx.x;
            const int jst = threadIdx.x >> 6;        // the source's sub-tile
            if (j < N && jst >= st0 && jst < st1) {
                for (int c = 0; c < 3; ++c) {
                    const float v = ((jpart[0][c][threadIdx.x] + jpart[1][c][threadIdx.x]) +
                                     jpart[2][c][threadIdx.x]) + jpart[3][c][threadIdx.x];
                    atomicAdd(&fix[c * stride + j], to_fixed((double)v, scale, status));
                }
            }
        }
        sx += (double)ax;
        sy += (double)ay;
        sz += (double)az;
    }
    if (i < N) {
        atomicAdd(&fix[i], to_fixed(sx, scale, status));
        atomicAdd(&fix[stride + i], to_fixed(sy, scale, status));
        atomicAdd(&fix[2 * stride + i], to_fixed(sz, scale, status));
    }
}

// R target tile rows I .. I + R - 1 against source tiles [J0, J1): each lane
// holds one target of every row, so one source (and one rotation of its
// reaction accumulator) serves R pairs.  When J0 == I the R x R block of the
// rows' own tiles is summed first by sym_item; the joint loop then starts at
// I + R, where every row is below the sources.
template <int BLOCK, int R, typename Pair>
__device__ __forceinline__ void sym_rows(const float* __restrict__ X, const float* __restrict__ Y,
                                         const float* __restrict__ Z, int N, int I, int J0, int J1,
                                         unsigned long long* __restrict__ fix, long long stride,
                                         double scale, int* status, float4 (*src)[128],
                                         float (*jpart)[3][BLOCK], const Pair& pair)
{
    if (J0 == I) {
        for (int r = 0; r < R; ++r)
            sym_item<BLOCK>(X, Y, Z, N, I + r, I + r, I + R, 0, 4, fix, stride, scale, status, src, jpart, pair);
        J0 = I + R;
    }
    if (J0 >= J1) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float xt[R], yt[R], zt[R];
    double sx[R], sy[R], sz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = (I + r) * BLOCK + threadIdx.x;
        xt[r] = X[i];
        yt[r] = Y[i];
        zt[r] = Z[i];
        sx[r] = sy[r] = sz[r] = 0.0;
    }
    for (int J = J0; J < J1; ++J) {
        const int j0 = J * BLOCK;
        __syncthreads();
        {
            const int st = threadIdx.x >> 6, l = threadIdx.x & 63;
            const float4 q = make_float4(X[j0 + threadIdx.x], Y[j0 + threadIdx.x], Z[j0 + threadIdx.x], 0.0f);
            src[st][l] = q;
            src[st][l + 64] = q;
        }
        __syncthreads();
        float ax[R], ay[R], az[R];
#pragma unroll
        for (int r = 0; r < R; ++r) ax[r] = ay[r] = az[r] = 0.0f;
        for (int st = 0; st < 4; ++st) {
            float jx = 0.0f, jy = 0.0f, jz = 0.0f;
            const float4* base = &src[st][lane];
#pragma unroll
            for (int k = 0; k < 64; ++k) {
                const float4 q = base[k];                     // source (lane + k) mod 64
                float dx[R], dy[R], dz[R], f[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    dx[r] = xt[r] - q.x;
                    dy[r] = yt[r] - q.y;
                    dz[r] = zt[r] - q.z;
                }
#pragma unroll
                for (int r = 0; r < R; ++r) f[r] = pair(dx[r], dy[r], dz[r]);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    ax[r] = fmaf(f[r], dx[r], ax[r]);
                    ay[r] = fmaf(f[r], dy[r], ay[r]);
                    az[r] = fmaf(f[r], dz[r], az[r]);
                    jx = fmaf(-f[r], dx[r], r == 0 ? rotate_down(jx) : jx);
                    jy = fmaf(-f[r], dy[r], r == 0 ? rotate_down(jy) : jy);
                    jz = fmaf(-f[r], dz[r], r == 0 ? rotate_down(jz) : jz);
                }
            }
            const int sid = st * 64 + ((lane + 63) & 63);
            jpart[wv][0][sid] = jx;
            jpart[wv][1][sid] = jy;
            jpart[wv][2][sid] = jz;
        }
        __syncthreads();
        const int j = j0 + threadIdx.x;
        if (j < N) {
            for (int c = 0; c < 3; ++c) {
                const float v = ((jpart[0][c][threadIdx.x] + jpart[1][c][threadIdx.x]) +
                                 jpart[2][c][threadIdx.x]) + jpart[3][c][threadIdx.x];
                atomicAdd(&fix[c * stride + j], to_fixed((double)v, scale, status));
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            sx[r] += (double)ax[r];
            sy[r] += (double)ay[r];
            sz[r] += (double)az[r];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = (I + r) * BLOCK + threadIdx.x;
        if (i < N) {
            atomicAdd(&fix[i], to_fixed(sx[r], scale, status));
            atomicAdd(&fix[stride + i], to_fixed(sy[r], scale, status));
            atomicAdd(&fix[2 * stride + i], to_fixed(sz[r], scale, status));
        }
    }
}

// One work item: rows == 1 is sym_item, rows == kSymRows is sym_rows.
template <int BLOCK, typename Pair>
__device__ __forceinline__ void sym_dispatch(const float* __restrict__ X, const float* __restrict__ Y,
                                             const float* __restrict__ Z, int N, int rows, int I, int J0,
                                             int J1, int st0, int st1, unsigned long long* __restrict__ fix,
                                             long long stride, double scale, int* status, float4 (*src)[128],
                                             float (*jpart)[3][BLOCK], const Pair& pair)
{
    if (rows == kSymRows)
        sym_rows<BLOCK, kSymRows>(X, Y, Z, N, I, J0, J1, fix, stride, scale, status, src, jpart, pair);
    else
        sym_item<BLOCK>(X, Y, Z, N, I, J0, J1, st0, st1, fix, stride, scale, status, src, jpart, pair);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kSymWaves, 8)))
void pair_sym_kernel(const float* __restrict__ xs, int Npad, int N, double scale,
                     const SymItem* __restrict__ items, unsigned long long* __restrict__ acc_fix,
                     Ctl* __restrict__ ctl)
{
    __shared__ float4 src[4][128];          // sub-tiles of 64 sources, each stored twice
    __shared__ float jpart[4][3][BLOCK];    // reactions per wave
    const SymItem it = items[blockIdx.x];
    sym_dispatch<BLOCK>(xs, xs + Npad, xs + 2 * Npad, N, it.rows, it.I, it.J0, it.J1, it.st0, it.st1, acc_fix,
                        Npad, scale, &ctl->status, src, jpart, PlainPair{});
}

}  // namespace odk
