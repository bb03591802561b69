// pairsym.hpp -- the all-pairs ion-ion sum with each pair evaluated once.
//
// The screened Coulomb force is antisymmetric, so the tile pair (I, J) of
// 256-ion target and source tiles also gives the reaction on the sources.
// Work items are runs of tiles J in [J0, J1) of one target tile row I
// (J >= I), longest first.  Within an item:
//   * the diagonal tile (J == I) is summed one-sided (each ordered pair);
//   * an off-diagonal tile is cut into four sub-tiles of 64 sources; lane l of
//     a wave pairs its target with source (l + k) mod 64 in step k, adds the
//     term to its own sum and subtracts it from a source accumulator that
//     moves one lane down each step (a wavefront rotate), so that after 64
//     steps every lane holds the reaction on one source, summed over the
//     wave's 64 targets in a fixed order; the four waves' sums are added in
//     LDS in a fixed order;
//   * reactions go to the sources' int64 fixed-point accumulators once per
//     tile pair, and the targets' sum once per item.
// Fixed-point integer addition is exact and commutative, so the totals do
// not depend on the order in which items run: results are deterministic.
// A per-ion epilogue kernel converts the totals, adds the grain, drive and
// confinement terms and the Eq. (1) sums (pair_epilogue), and clears the
// accumulators for the next step.
#pragma once

#include "kernels.hpp"

namespace odk {

// The accumulators hold the raw sums (1 + r) e^-r / r^3 d times a per-system
// power of two, PairArgs::sym_scale, set by the host from the ion density so
// that the resolution stays near 1e-8 of a typical sum (dominated by the
// nearest neighbours, ~ n^(2/3)) while the int64 range keeps a margin of
// about 1e13 for close pairs.

// rows == 1: target tile row I against source tiles [J0, J1) (sym_item);
// rows == 2: target tile rows I and I + 1 together (sym_item2).
struct SymItem {
    int I, J0, J1, rows;
};

// One pair term (1 + r) e^-r / r^3 for the difference d.
__device__ __forceinline__ float sym_f(float dx, float dy, float dz)
{
    const float kNegLog2e = -1.4426950408889634f;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ri;
    const float e = __builtin_amdgcn_exp2f(r * kNegLog2e);
    const float ri2 = ri * ri;
    return fmaf(ri2, ri, ri2) * e;
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
// I against source tiles [J0, J1), J0 >= I.  Reactions go to
// fix[c * stride + j], the targets' sums to fix[c * stride + i] (indices
// local to the system).  pair(d) is the scalar f of the term f d.
template <int BLOCK, typename Pair>
__device__ __forceinline__ void sym_item(const float* __restrict__ X, const float* __restrict__ Y,
                                         const float* __restrict__ Z, int N, int I, int J0, int J1,
                                         unsigned long long* __restrict__ fix, long long stride,
                                         double scale, int* status, float4 (*src)[128],
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
            for (int k = 0; k < BLOCK; ++k) {
                const float4 q = src[k >> 6][k & 63];
                const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
                float f = pair(dx, dy, dz);
                f = (k == (int)threadIdx.x) ? 0.0f : f;
                ax = fmaf(f, dx, ax);
                ay = fmaf(f, dy, ay);
                az = fmaf(f, dz, az);
            }
        } else {
            for (int st = 0; st < 4; ++st) {
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
            if (j < N) {
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

// Two target tile rows Ia = I and Ib = I + 1 against source tiles [J0, J1):
// each lane holds one target of each row, so one source (and one rotation
// of its reaction accumulator) serves two pairs.  The 2 x 2 block of the rows'
// own tiles is summed by sym_item first when J0 == I; the joint loop then
// starts at I + 2, where both rows are below the sources.
template <int BLOCK, typename Pair>
__device__ __forceinline__ void sym_item2(const float* __restrict__ X, const float* __restrict__ Y,
                                          const float* __restrict__ Z, int N, int I, int J0, int J1,
                                          unsigned long long* __restrict__ fix, long long stride,
                                          double scale, int* status, float4 (*src)[128],
                                          float (*jpart)[3][BLOCK], const Pair& pair)
{
    if (J0 == I) {
        sym_item<BLOCK>(X, Y, Z, N, I, I, I + 2, fix, stride, scale, status, src, jpart, pair);
        sym_item<BLOCK>(X, Y, Z, N, I + 1, I + 1, I + 2, fix, stride, scale, status, src, jpart, pair);
        J0 = I + 2;
    }
    if (J0 >= J1) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ia = I * BLOCK + threadIdx.x, ib = ia + BLOCK;
    const float xa = X[ia], ya = Y[ia], za = Z[ia];
    const float xb = X[ib], yb = Y[ib], zb = Z[ib];
    double sxa = 0.0, sya = 0.0, sza = 0.0, sxb = 0.0, syb = 0.0, szb = 0.0;
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
        float axa = 0.0f, aya = 0.0f, aza = 0.0f, axb = 0.0f, ayb = 0.0f, azb = 0.0f;
        for (int st = 0; st < 4; ++st) {
            float jx = 0.0f, jy = 0.0f, jz = 0.0f;
            const float4* base = &src[st][lane];
#pragma unroll 8
            for (int k = 0; k < 64; ++k) {
                const float4 q = base[k];                     // source (lane + k) mod 64
                const float dxa = xa - q.x, dya = ya - q.y, dza = za - q.z;
                const float dxb = xb - q.x, dyb = yb - q.y, dzb = zb - q.z;
                const float fa = pair(dxa, dya, dza);
                const float fb = pair(dxb, dyb, dzb);
                axa = fmaf(fa, dxa, axa);
                aya = fmaf(fa, dya, aya);
                aza = fmaf(fa, dza, aza);
                axb = fmaf(fb, dxb, axb);
                ayb = fmaf(fb, dyb, ayb);
                azb = fmaf(fb, dzb, azb);
                jx = fmaf(-fb, dxb, fmaf(-fa, dxa, rotate_down(jx)));
                jy = fmaf(-fb, dyb, fmaf(-fa, dya, rotate_down(jy)));
                jz = fmaf(-fb, dzb, fmaf(-fa, dza, rotate_down(jz)));
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
        sxa += (double)axa; sya += (double)aya; sza += (double)aza;
        sxb += (double)axb; syb += (double)ayb; szb += (double)azb;
    }
    if (ia < N) {
        atomicAdd(&fix[ia], to_fixed(sxa, scale, status));
        atomicAdd(&fix[stride + ia], to_fixed(sya, scale, status));
        atomicAdd(&fix[2 * stride + ia], to_fixed(sza, scale, status));
    }
    if (ib < N) {
        atomicAdd(&fix[ib], to_fixed(sxb, scale, status));
        atomicAdd(&fix[stride + ib], to_fixed(syb, scale, status));
        atomicAdd(&fix[2 * stride + ib], to_fixed(szb, scale, status));
    }
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8, 8)))
void pair_sym_kernel(const float* __restrict__ xs, int Npad, int N, double scale,
                     const SymItem* __restrict__ items, unsigned long long* __restrict__ acc_fix,
                     Ctl* __restrict__ ctl)
{
    __shared__ float4 src[4][128];          // sub-tiles of 64 sources, each stored twice
    __shared__ float jpart[4][3][BLOCK];    // reactions per wave
    const SymItem it = items[blockIdx.x];
    if (it.rows == 2)
        sym_item2<BLOCK>(xs, xs + Npad, xs + 2 * Npad, N, it.I, it.J0, it.J1, acc_fix, Npad, scale,
                         &ctl->status, src, jpart, PlainPair{});
    else
        sym_item<BLOCK>(xs, xs + Npad, xs + 2 * Npad, N, it.I, it.J0, it.J1, acc_fix, Npad, scale,
                        &ctl->status, src, jpart, PlainPair{});
}

// Per ion: total of the pair sums, then the terms of pair_epilogue; clears
// the accumulators (every slot of the Npad planes).
__global__ __launch_bounds__(256) void pair_sym_epilogue(const float* __restrict__ xs,
                                                         unsigned long long* __restrict__ acc_fix,
                                                         float* __restrict__ acc, PairArgs p,
                                                         DustSet ds, Ctl* __restrict__ ctl)
{
    __shared__ double red[4][kMaxDust][3];
    const int Npad = p.Npad;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool live = i < p.N;
    const float xi = xs[i], yi = xs[Npad + i], zi = xs[2 * Npad + i];
    double s[3];
    for (int c = 0; c < 3; ++c) {
        unsigned long long* a = &acc_fix[(long long)c * Npad + i];
        s[c] = live ? from_fixed(*a, p.sym_scale) : 0.0;
        *a = 0ull;
    }
    pair_epilogue<256>(xi, yi, zi, i, live, p.Cd * s[0], p.Cd * s[1], p.Cd * s[2], true, p, ds, ctl,
                       acc, acc + Npad, acc + 2 * Npad, red);
}

}  // namespace odk
