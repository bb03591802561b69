// batch.hpp -- kernels that advance many independent dust systems together.
//
// All systems share one structure-of-arrays arena: plane c of x holds every
// system's ions, system s at [off_s, off_s + Npad_s) (Npad_s a multiple of
// 256).  Per-system constants live in a device table of SysDesc.  The pair
// forces run as a list of work items (system, 256-ion target block, source
// range, split index) pulled from an atomic queue by a persistent grid, most
// expensive first; a system whose sources are split over several items
// writes partial accelerations to separate planes that the push adds in a
// fixed order, so results do not depend on scheduling.
#pragma once

#include "kernels.hpp"
#include "pairsym.hpp"

namespace odk {

struct SysDesc {
    long long off;          // first ion of the system in the arena
    int nsplit;             // source splits of the pair sum (partial planes)
    int blk0;               // first push block of the system
    PairArgs pa;
    PushArgs pu;
    DustSet ds;
    FinalArgs fa;
};

struct PairItem {
    int sys, i0, jb, je, split, pad_[3];
};

struct BatchCtl {
    unsigned int queue;                 // next pair work item
    unsigned int pad_;
    unsigned long long n_lost[kSlots];  // lost-list segment lengths
    int status;
    int pad2_[11];
};

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Pair forces of the whole batch.  persistent != 0: a fixed grid pulls items
// from bc->queue until the list is exhausted (every block leaves when the
// counter passes n_items); else block b does item b.
template <int BLOCK, int TJ>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8, 8)))
void pair_batch_kernel(const float* __restrict__ xs,
                                                           float* __restrict__ acc,
                                                           long long plane, const SysDesc* sys,
                                                           Ctl* __restrict__ ctls,
                                                           const PairItem* __restrict__ items,
                                                           int n_items, BatchCtl* bc,
                                                           int persistent)
{
    __shared__ float4 tile[TJ];
    __shared__ double red[BLOCK / 64][kMaxDust][3];
    __shared__ int cur;
    int it = blockIdx.x;
    for (;;) {
        if (persistent) {
            if (threadIdx.x == 0) cur = (int)atomicAdd(&bc->queue, 1u);
            __syncthreads();
            it = uniform_int(cur);
            __syncthreads();
        }
        if (it >= n_items) break;
        const int s = uniform_int(items[it].sys);
        const int i0 = uniform_int(items[it].i0);
        const int jb = uniform_int(items[it].jb);
        const int je = uniform_int(items[it].je);
        const int split = uniform_int(items[it].split);
        const SysDesc& S = sys[s];
        const long long off = S.off;
        const float* X = xs + off;
        float* o = acc + (long long)split * 3 * plane + off;
        pair_block_f32<BLOCK, TJ>(X, X + plane, X + 2 * plane, i0, jb, je, S.pa, S.ds, ctls + s, o,
                                  o + plane, o + 2 * plane, split == 0, tile, red);
        if (!persistent) break;
    }
}

// Symmetric pair sums of the batch (each unordered pair once, see
// pairsym.hpp): item = (system, target tile row, source tile run); int64
// fixed-point totals in fix (planes `plane` apart, system at its offset).
struct SymBatchItem {
    int sys, I, J0, J1, rows, pad_[3];
};

template <int BLOCK, int TJ>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kSymWaves, 8)))
void pair_sym_batch_kernel(const float* __restrict__ xs, long long plane, const SysDesc* sys,
                           Ctl* __restrict__ ctls, const SymBatchItem* __restrict__ items,
                           unsigned long long* __restrict__ fix)
{
    static_assert(BLOCK == TJ, "square tiles");
    __shared__ float4 src[4][128];
    __shared__ float jpart[4][3][BLOCK];
    const SymBatchItem it = items[blockIdx.x];
    const int s = uniform_int(it.sys);
    const long long off = sys[s].off;
    const float* X = xs + off;
    const int I = uniform_int(it.I), J0 = uniform_int(it.J0), J1 = uniform_int(it.J1);
    sym_dispatch<BLOCK>(X, X + plane, X + 2 * plane, sys[s].pa.N, uniform_int(it.rows), I, J0, J1, fix + off,
                        plane, sys[s].pa.sym_scale, &ctls[s].status, src, jpart, PlainPair{});
}

// Per ion of every system (block b belongs to system blk_sys[b]): converts
// the fixed-point totals, adds the pair_epilogue terms, clears the totals.
__global__ __launch_bounds__(256) void pair_sym_batch_epilogue(const float* __restrict__ xs,
                                                               float* __restrict__ acc, long long plane,
                                                               unsigned long long* __restrict__ fix,
                                                               const SysDesc* sys, Ctl* __restrict__ ctls,
                                                               const int* __restrict__ blk_sys)
{
    __shared__ double red[4][kMaxDust][3];
    const int s = uniform_int(blk_sys[blockIdx.x]);
    const SysDesc& S = sys[s];
    const long long off = S.off;
    const int i = (blockIdx.x - S.blk0) * 256 + threadIdx.x;
    const bool live = i < S.pa.N;
    const float* X = xs + off;
    const float xi = X[i], yi = X[plane + i], zi = X[2 * plane + i];
    double v[3];
    for (int c = 0; c < 3; ++c) {
        unsigned long long* a = &fix[c * plane + off + i];
        v[c] = live ? from_fixed(*a, S.pa.sym_scale) : 0.0;
        *a = 0ull;
    }
    float* o = acc + off;
    pair_epilogue<256>(xi, yi, zi, i, live, S.pa.Cd * v[0], S.pa.Cd * v[1], S.pa.Cd * v[2], true, S.pa,
                       S.ds, ctls + s, o, o + plane, o + 2 * plane, red);
}

// Push of the whole batch: block b belongs to system blk_sys[b].
__global__ __launch_bounds__(256) void push_batch_kernel(float* __restrict__ xs,
                                                         float* __restrict__ vs,
                                                         const float* __restrict__ as,
                                                         long long plane, uint8_t* __restrict__ ev,
                                                         int2* __restrict__ lost_list,
                                                         const SysDesc* sys, Ctl* __restrict__ ctls,
                                                         const int* __restrict__ blk_sys,
                                                         BatchCtl* bc)
{
    const int s = uniform_int(blk_sys[blockIdx.x]);
    const SysDesc& S = sys[s];
    Ctl* ctl = ctls + s;
    const long long off = S.off;
    const int i = (blockIdx.x - S.blk0) * 256 + threadIdx.x;
    const uint64_t n = (uint64_t)ctl->step;
    bool coll = false, lost = false;
    uint8_t code = kEvNone;
    if (i < S.pu.N) {
        float* X = xs + off;
        float* V = vs + off;
        const float* A = as + off;
        push_ion<float>(X, X + plane, X + 2 * plane, V, V + plane, V + 2 * plane, A, A + plane,
                        A + 2 * plane, 3 * plane, S.nsplit, i, n, S.pu, S.ds, ctl, code, coll, lost);
        ev[off + i] = code | (coll ? kEvCollBit : 0);
    }
    const long long at = wave_tally(ctl, code, coll, lost, bc->n_lost, seg_cap(gridDim.x));
    if (lost) lost_list[at] = make_int2(s, i);
}

// Block b walks segment b mod kSlots of the lost list (grid: a multiple of
// kSlots); cap: segment capacity of the push grid.
__global__ __launch_bounds__(64) void reinject_batch_kernel(float* __restrict__ xs,
                                                            float* __restrict__ vs, long long plane,
                                                            const int2* __restrict__ lost_list,
                                                            long long cap, const SysDesc* sys,
                                                            Ctl* __restrict__ ctls, BatchCtl* bc)
{
    const int slot = blockIdx.x % kSlots, part = blockIdx.x / kSlots, parts = gridDim.x / kSlots;
    const long long cnt = (long long)bc->n_lost[slot];
    const int2* seg = lost_list + slot * cap;
    for (long long k = part * 64 + threadIdx.x; k < cnt; k += (long long)parts * 64) {
        const int2 e = seg[k];
        const SysDesc& S = sys[e.x];
        float* X = xs + S.off;
        float* V = vs + S.off;
        reinject_ion<float>(X, X + plane, X + 2 * plane, V, V + plane, V + 2 * plane, e.y,
                            (uint64_t)ctls[e.x].step, S.pu);
    }
}

// One wave per system; block 0 also rewinds the batch's queue and list.
__global__ __launch_bounds__(64) void finalize_batch_kernel(const SysDesc* sys,
                                                            Ctl* __restrict__ ctls, BatchCtl* bc)
{
    __shared__ double Qs[kMaxDust];
    const SysDesc& S = sys[blockIdx.x];
    finalize_sys(S.fa, S.ds, ctls + blockIdx.x, Qs);
    if (blockIdx.x == 0) {
        bc->n_lost[threadIdx.x] = 0ull;     // blockDim.x == kSlots
        if (threadIdx.x == 0) bc->queue = 0u;
    }
}

__global__ __launch_bounds__(256) void init_batch_kernel(float* __restrict__ xs,
                                                         float* __restrict__ vs,
                                                         float* __restrict__ as, long long plane,
                                                         int max_split, const SysDesc* sys,
                                                         Ctl* __restrict__ ctls,
                                                         const int* __restrict__ blk_sys)
{
    const int s = uniform_int(blk_sys[blockIdx.x]);
    const SysDesc& S = sys[s];
    const long long off = S.off;
    const int i = (blockIdx.x - S.blk0) * 256 + threadIdx.x;
    float* X = xs + off;
    float* V = vs + off;
    init_ion<float>(X, X + plane, X + 2 * plane, V, V + plane, V + 2 * plane, i, S.pu, S.ds,
                    ctls + s);
    for (int k = 0; k < max_split; ++k)
        for (int c = 0; c < 3; ++c) as[(long long)(3 * k + c) * plane + off + i] = 0.0f;
}

}  // namespace odk
