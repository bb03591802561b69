// cutoff.hpp -- ion-ion forces with a cutoff distance and switching function
// (the paper's option for long domains, Section 4).
//
// The pair energy phi(r) = C e^-r / r is multiplied by the smooth step
// S(r) = 1 - 6x^5 + 15x^4 - 10x^3, x = clamp((r - r_sw) / (r_cut - r_sw), 0, 1),
// and the force is -d(phi S)/dr; S and S' vanish from r_cut on, so pairs
// beyond the cutoff contribute exactly zero without a branch.
//
// Every step the ions are binned into slabs along z (width w, about r_cut / 16,
// or r_cut / 8 in domains long enough to pass kMaxSlabs)
// and sorted by slab with a stable counting sort (so the order, and with it every
// floating-point sum, is deterministic):
//   slab_count_kernel    slab of each ion; per-block slab histogram
//   slab_scan_kernel     per slab, exclusive scan over blocks; slab totals
//   slab_start_kernel    exclusive scan of the slab totals
//   slab_scatter_kernel  sorted copy of the positions and their ion indices
// Pairs are then taken once each (as in pairsym.hpp): a block of 256
// consecutive sorted ions (tile I) meets the sorted tiles J = I .. J1 - 1,
// where J1 ends at the last source of the slabs within `reach` =
// ceil(r_cut / w) slabs above its own (pair_cut_kernel).  A pair within r_cut
// with its lower member in tile I has its upper member there, since sorted
// order puts it at most `reach` slabs higher.  The totals go to int64
// fixed-point accumulators indexed by sorted slot; pair_cut_epilogue writes
// the accelerations back to the ions' own slots.
#pragma once

#include "kernels.hpp"
#include "pairsym.hpp"

namespace odk {

constexpr int kMaxSlabs = 1024;

struct CutArgs {
    int nslab;        // slabs along z
    int nblk;         // blocks of 256 ions (sort granularity)
    int reach;        // slabs on either side that can hold a source within r_cut
    int pad_;
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

// The switched pair term as a functor for sym_item.
struct SwitchedPair {
    float rsw, inv_sw, dS_c;
    __device__ __forceinline__ float operator()(float dx, float dy, float dz) const
    {
        const float kNegLog2e = -1.4426950408889634f;
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float r = r2 * ri;
        const float e = __builtin_amdgcn_exp2f(r * kNegLog2e);
        const float x = __builtin_amdgcn_fmed3f((r - rsw) * inv_sw, 0.0f, 1.0f);
        const float x2 = x * x;
        const float S = fmaf(x2 * x, fmaf(fmaf(-6.0f, x, 15.0f), x, -10.0f), 1.0f);
        const float u = fmaf(-x, x, x);              // x (1 - x)
        const float dS = dS_c * u * u;               // S'(r) = -30 x^2 (1 - x)^2 / (r_cut - r_sw)
        const float g = fmaf(r, S, S) - r * dS;      // (1 + r) S - r S'
        return (ri * ri * ri) * (e * g);
    }
};

// Switched forces, each pair once: block b takes sorted tile I = b against
// the tiles up to the end of the slabs within reach above its last ion; the
// sums go to fix (planes Npad apart, sorted slots).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8, 8)))
void pair_cut_kernel(const float* __restrict__ xs_sorted, const int* __restrict__ start,
                     unsigned long long* __restrict__ fix, PairArgs p, CutArgs c,
                     Ctl* __restrict__ ctl)
{
    __shared__ float4 src[4][128];
    __shared__ float jpart[4][3][BLOCK];
    if (!p.ion_ion) return;
    const int Npad = p.Npad, N = p.N;
    const float* Z = xs_sorted + 2 * Npad;
    const int I = blockIdx.x;
    const int s_hi = slab_of_z(Z[min((I + 1) * BLOCK, N) - 1], c);
    const int je = start[min(s_hi + c.reach + 1, c.nslab)];
    const int J1 = (je + BLOCK - 1) / BLOCK;
    const SwitchedPair pair{c.rsw, c.inv_sw, -30.0f * c.inv_sw};
    sym_item<BLOCK>(xs_sorted, xs_sorted + Npad, Z, N, I, I, J1, 0, 4, fix, Npad, p.sym_scale, &ctl->status,
                    src, jpart, pair);
}

// Per sorted slot: converts the totals, adds the pair_epilogue terms and
// writes the acceleration to the ion's own slot; clears the totals.
__global__ __launch_bounds__(256) void pair_cut_epilogue(const float* __restrict__ xs_sorted,
                                                         const int* __restrict__ idx,
                                                         unsigned long long* __restrict__ fix,
                                                         float* __restrict__ acc, PairArgs p,
                                                         DustSet ds, Ctl* __restrict__ ctl)
{
    __shared__ double red[4][kMaxDust][3];
    const int Npad = p.Npad;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool live = i < p.N;
    const float xi = xs_sorted[i], yi = xs_sorted[Npad + i], zi = xs_sorted[2 * Npad + i];
    double v[3];
    for (int c = 0; c < 3; ++c) {
        unsigned long long* a = &fix[(long long)c * Npad + i];
        v[c] = live ? from_fixed(*a, p.sym_scale) : 0.0;
        *a = 0ull;
    }
    pair_epilogue<256>(xi, yi, zi, live ? idx[i] : 0, live, p.Cd * v[0], p.Cd * v[1], p.Cd * v[2], true,
                       p, ds, ctl, acc, acc + Npad, acc + 2 * Npad, red);
}

}  // namespace odk
