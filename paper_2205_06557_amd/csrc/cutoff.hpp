// cutoff.hpp -- ion-ion forces with a cutoff distance and switching function
// (the paper's option for long domains, Section 4).
//
// The pair energy phi(r) = C e^-r / r is multiplied by the smooth step
// S(r) = 1 - 6x^5 + 15x^4 - 10x^3, x = clamp((r - r_sw) / (r_cut - r_sw), 0, 1),
// and the force is -d(phi S)/dr; S and S' vanish from r_cut on, so pairs
// beyond the cutoff contribute exactly zero without a branch.
//
// Every step the ions are binned into slabs along z of width >= r_cut and
// sorted by slab with a stable counting sort (so the order, and with it every
// floating-point sum, is deterministic):
//   slab_count_kernel    slab of each ion; per-block slab histogram
//   slab_scan_kernel     per slab, exclusive scan over blocks; slab totals
//   slab_start_kernel    exclusive scan of the slab totals
//   slab_scatter_kernel  sorted copy of the positions and their ion indices
// A block of 256 consecutive sorted targets then meets only the sources of
// its own slabs and one slab on either side (pair_cut_kernel), and writes
// the accelerations back to the ions' own slots.
#pragma once

#include "kernels.hpp"

namespace odk {

constexpr int kMaxSlabs = 1024;

struct CutArgs {
    int nslab;        // slabs along z
    int nblk;         // blocks of 256 ions (sort granularity)
    float z0;         // lower end of the domain, -H/2
    float inv_w;      // 1 / slab width
    float rsw;        // start of the switching interval
    float inv_sw;     // 1 / (r_cut - r_sw)
};

__device__ __forceinline__ int slab_of_z(float z, const CutArgs& c)
{
    const int s = (int)((z - c.z0) * c.inv_w);
    return min(max(s, 0), c.nslab - 1);
}

// table[s * nblk + b] = number of ions of block b in slab s.
__global__ __launch_bounds__(256) void slab_count_kernel(const float* __restrict__ Z, int N,
                                                         CutArgs c, int* __restrict__ slab,
                                                         int* __restrict__ table)
{
    __shared__ int hist[kMaxSlabs];
    for (int s = threadIdx.x; s < c.nslab; s += 256) hist[s] = 0;
    __syncthreads();
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < N) {
        const int s = slab_of_z(Z[i], c);
        slab[i] = s;
        atomicAdd(&hist[s], 1);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < c.nslab; s += 256) table[(long long)s * c.nblk + blockIdx.x] = hist[s];
}

// One block per slab: table row s becomes its exclusive prefix sum over
// blocks; total[s] receives the row sum.
__global__ __launch_bounds__(256) void slab_scan_kernel(int* __restrict__ table, int nblk,
                                                        int* __restrict__ total)
{
    __shared__ int wsum[4];
    __shared__ int carry;
    int* row = table + (long long)blockIdx.x * nblk;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int b0 = 0; b0 < nblk; b0 += 256) {
        const int b = b0 + threadIdx.x;
        const int v = b < nblk ? row[b] : 0;
        // inclusive scan in the wave
        int x = v;
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        int before = carry;
        for (int w = 0; w < wv; ++w) before += wsum[w];
        if (b < nblk) row[b] = before + x - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) total[blockIdx.x] = carry;
}

// start[s] = sum of total[0..s), s = 0..nslab (one block of 1024 threads).
__global__ __launch_bounds__(1024) void slab_start_kernel(const int* __restrict__ total, int nslab,
                                                          int* __restrict__ start)
{
    __shared__ int buf[kMaxSlabs];
    const int t = threadIdx.x;
    buf[t] = t < nslab ? total[t] : 0;
    __syncthreads();
    for (int d = 1; d < kMaxSlabs; d <<= 1) {
        const int y = t >= d ? buf[t - d] : 0;
        __syncthreads();
        buf[t] += y;
        __syncthreads();
    }
    if (t < nslab) start[t + 1] = buf[t];
    if (t == 0) start[0] = 0;
}

// Sorted copy: ion i of block b goes to start[s] + table[s][b] + (number of
// ions of slab s before it in block b), which keeps ion order within a slab.
// The waves of the block take their turns; within a wave, lanes of one slab
// are ranked with a ballot.
__global__ __launch_bounds__(256) void slab_scatter_kernel(const float* __restrict__ X,
                                                           const float* __restrict__ Y,
                                                           const float* __restrict__ Z, int N,
                                                           CutArgs c, const int* __restrict__ slab,
                                                           const int* __restrict__ table,
                                                           const int* __restrict__ start,
                                                           float* __restrict__ Xs,
                                                           float* __restrict__ Ys,
                                                           float* __restrict__ Zs,
                                                           int* __restrict__ idx)
{
    __shared__ int run[kMaxSlabs];
    for (int s = threadIdx.x; s < c.nslab; s += 256) run[s] = 0;
    __syncthreads();
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool live = i < N;
    const int s = live ? slab[i] : -1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int w = 0; w < 4; ++w) {
        if (wv == w) {
            unsigned long long todo = __ballot(live);
            while (todo) {
                const int leader = __ffsll((long long)todo) - 1;
                const int key = __shfl(s, leader, 64);
                const unsigned long long same = __ballot(live && s == key);
                if (live && s == key) {
                    const int rank = __popcll(same & below);
                    const int pos = start[s] + table[(long long)s * c.nblk + blockIdx.x] + run[s] + rank;
                    Xs[pos] = X[i];
                    Ys[pos] = Y[i];
                    Zs[pos] = Z[i];
                    idx[pos] = i;
                }
                if (lane == leader) run[key] += __popcll(same);
                todo &= ~same;
            }
        }
        __syncthreads();
    }
}

// One switched pair term added to (ax, ay, az): f d with
// f = e^-r [(1 + r) S - r S'] / r^3, i.e. -d(phi S)/dr / (C r); skip zeroes it.
__device__ __forceinline__ void cut_pair(float xi, float yi, float zi, float4 q, float rsw,
                                         float inv_sw, float dS_c, float& ax, float& ay, float& az,
                                         bool skip)
{
    const float kNegLog2e = -1.4426950408889634f;
    const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ri;
    const float e = __builtin_amdgcn_exp2f(r * kNegLog2e);
    const float x = __builtin_amdgcn_fmed3f((r - rsw) * inv_sw, 0.0f, 1.0f);
    const float x2 = x * x;
    const float S = fmaf(x2 * x, fmaf(fmaf(-6.0f, x, 15.0f), x, -10.0f), 1.0f);
    const float u = fmaf(-x, x, x);                  // x (1 - x)
    const float dS = dS_c * u * u;                   // S'(r) = -30 x^2 (1 - x)^2 / (r_cut - r_sw)
    const float g = fmaf(r, S, S) - r * dS;          // (1 + r) S - r S'
    float f = (ri * ri * ri) * (e * g);
    f = skip ? 0.0f : f;
    ax = fmaf(f, dx, ax);
    ay = fmaf(f, dy, ay);
    az = fmaf(f, dz, az);
}

// Forces with the cutoff: block b takes sorted targets [256 b, 256 b + 256)
// against the sorted sources of slabs s_lo - 1 .. s_hi + 1, in tiles of TJ
// (entries past the range are parked far away and contribute zero).
template <int BLOCK, int TJ>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8, 8)))
void pair_cut_kernel(const float* __restrict__ xs_sorted, const int* __restrict__ idx,
                     const int* __restrict__ start, float* __restrict__ acc, PairArgs p,
                     CutArgs c, DustSet ds, Ctl* __restrict__ ctl)
{
    __shared__ float4 tile[TJ];
    __shared__ double red[BLOCK / 64][kMaxDust][3];
    const int Npad = p.Npad, N = p.N;
    const float* X = xs_sorted;
    const float* Y = xs_sorted + Npad;
    const float* Z = xs_sorted + 2 * Npad;
    const int i0 = blockIdx.x * BLOCK;
    const int i = i0 + threadIdx.x;
    const bool live = i < N;
    const float xi = X[i], yi = Y[i], zi = Z[i];
    const int s_lo = slab_of_z(Z[i0], c);
    const int s_hi = slab_of_z(Z[min(i0 + BLOCK, N) - 1], c);
    const int jb = start[max(s_lo - 1, 0)];
    const int je = start[min(s_hi + 2, c.nslab)];
    const float rsw = c.rsw, inv_sw = c.inv_sw;
    const float dS_c = -30.0f * inv_sw;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    if (p.ion_ion) {
        for (int j0 = jb; j0 < je; j0 += TJ) {
            __syncthreads();
            for (int t = threadIdx.x; t < TJ; t += BLOCK) {
                const int j = j0 + t;
                tile[t] = j < je ? make_float4(X[j], Y[j], Z[j], 0.0f)
                                 : make_float4(1.0e18f, 1.0e18f, 1.0e18f, 0.0f);
            }
            __syncthreads();
            float ax = 0.0f, ay = 0.0f, az = 0.0f;
            if (i0 + BLOCK <= j0 || j0 + TJ <= i0) {
#pragma unroll 4
                for (int k = 0; k < TJ; ++k)
                    cut_pair(xi, yi, zi, tile[k], rsw, inv_sw, dS_c, ax, ay, az, false);
            } else {
                const int kself = i - j0;      // the target's own entry
                for (int k = 0; k < TJ; ++k)
                    cut_pair(xi, yi, zi, tile[k], rsw, inv_sw, dS_c, ax, ay, az, k == kself);
            }
            sx += (double)ax;
            sy += (double)ay;
            sz += (double)az;
        }
    }
    pair_epilogue<BLOCK>(xi, yi, zi, live ? idx[i] : 0, live, p.Cd * sx, p.Cd * sy, p.Cd * sz, true,
                         p, ds, ctl, acc, acc + Npad, acc + 2 * Npad, red);
}

}  // namespace odk
