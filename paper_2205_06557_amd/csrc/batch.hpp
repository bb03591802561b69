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

struct alignas(128) BatchCtl {
    unsigned int lost_seg[kSlots * kPad32];   // lost-list segment lengths (all systems), [s * kPad32]
    unsigned int queue;                 // next pair work item
    unsigned int lost_ticket;           // reinjection blocks that have finished
    int status;
    int pad2_[29];
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
// pairsym.hpp): item = (system, target tile rows, source tile run); int64
// fixed-point totals in fix (planes `plane` apart, system at its offset).
// The items are ordered most work first.  persistent != 0: a grid of about
// one resident wave of blocks pulls items from bc->queue (the longest-first
// greedy schedule, taken by whichever block frees up first) until the list is
// exhausted; else block b does item b and the hardware dispatcher hands out
// blocks in index order.  The totals are integers, so both give the same sums.
struct SymBatchItem {
    int sys, I, J0, J1, rows, st0, st1, pad_;
};

template <int BLOCK>
__device__ __forceinline__ void sym_batch_item(const float* __restrict__ xs, long long plane, const SysDesc* sys,
                                               Ctl* __restrict__ ctls, const SymBatchItem& it,
                                               unsigned long long* __restrict__ fix, float4 (*src)[128],
                                               float (*jpart)[3][BLOCK])
{
    const int s = uniform_int(it.sys);
    const long long off = sys[s].off;
    const float* X = xs + off;
    const int I = uniform_int(it.I), J0 = uniform_int(it.J0), J1 = uniform_int(it.J1);
    sym_dispatch<BLOCK>(X, X + plane, X + 2 * plane, sys[s].pa.N, uniform_int(it.rows), I, J0, J1,
                        uniform_int(it.st0), uniform_int(it.st1), fix + off, plane, sys[s].pa.sym_scale,
                        &ctls[s].status, src, jpart, PlainPair{});
}

template <int BLOCK, int TJ, bool PERSISTENT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kSymWaves, 8)))
void pair_sym_batch_kernel(const float* __restrict__ xs, long long plane, const SysDesc* sys,
                           Ctl* __restrict__ ctls, const SymBatchItem* __restrict__ items, int n_items,
                           unsigned long long* __restrict__ fix, BatchCtl* bc)
{
    static_assert(BLOCK == TJ, "square tiles");
    __shared__ float4 src[4][128];
    __shared__ float jpart[4][3][BLOCK];
    if (!PERSISTENT) {
        sym_batch_item<BLOCK>(xs, plane, sys, ctls, items[blockIdx.x], fix, src, jpart);
        return;
    }
    __shared__ int cur;
    for (;;) {
        if (threadIdx.x == 0) cur = (int)atomicAdd(&bc->queue, 1u);
        __syncthreads();
        const int k = uniform_int(cur);
        __syncthreads();
        if (k >= n_items) break;
        sym_batch_item<BLOCK>(xs, plane, sys, ctls, items[k], fix, src, jpart);
    }
}

// The per-ion tail of the step for every system (block b belongs to system
// blk_sys[b]; see tail_block): FIX for the symmetric pair sums (totals in
// fix), else the one-sided kernel's acceleration planes.  Block 0 also
// rewinds the pair kernel's work queue (that kernel has finished).
template <bool FIX>
__global__ __launch_bounds__(256) void step_tail_batch_kernel(float* __restrict__ xs, float* __restrict__ vs,
                                                              float* __restrict__ as, long long plane,
                                                              unsigned long long* __restrict__ fix,
                                                              uint8_t* __restrict__ ev, const SysDesc* sys,
                                                              Ctl* __restrict__ ctls,
                                                              const int* __restrict__ blk_sys, BatchCtl* bc,
                                                              int2* __restrict__ lost)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) bc->queue = 0u;
    const int s = uniform_int(blk_sys[blockIdx.x]);
    const SysDesc& S = sys[s];
    const long long off = S.off;
    float* X = xs + off;
    float* V = vs + off;
    float* A = as + off;
    tail_block<float, FIX>(X, X + plane, X + 2 * plane, V, V + plane, V + 2 * plane, A, A + plane, A + 2 * plane,
                           3 * plane, S.nsplit, FIX ? fix + off : nullptr, plane, ev + off,
                           (blockIdx.x - S.blk0) * 256, S.pa.Npad / 256, S.pa, S.pu, S.ds, S.fa, ctls + s, s,
                           LostList{bc->lost_seg, &bc->lost_ticket, lost, lost_cap(gridDim.x)});
}

// Reinjection of the batch's listed ions (system, ion).
struct BatchSystems {
    float* xs;
    float* vs;
    long long plane;
    const SysDesc* sys;
    const Ctl* ctls;
    __device__ void operator()(int s, float*& X, float*& V, const PushArgs*& p, const Ctl*& c,
                               long long& P) const
    {
        X = xs + sys[s].off; V = vs + sys[s].off; p = &sys[s].pu; c = ctls + s; P = plane;
    }
};

__global__ __launch_bounds__(64) void reinject_batch_kernel(float* __restrict__ xs, float* __restrict__ vs,
                                                            long long plane, const SysDesc* sys,
                                                            const Ctl* __restrict__ ctls, BatchCtl* bc,
                                                            int2* __restrict__ lost, long long cap)
{
    reinject_list<float>(LostList{bc->lost_seg, &bc->lost_ticket, lost, cap}, BatchSystems{xs, vs, plane, sys, ctls});
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
