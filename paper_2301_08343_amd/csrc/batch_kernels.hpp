// Batched substep kernels: many independent contacts advanced by one launch
// per phase. A launch's work items are (contact, grid block) pairs; each
// workgroup loads its contact's descriptor and runs the same block-level code
// as the single-contact kernels. The indenter of every contact and substep is
// tabulated on the device, and the substep index lives in device memory, so a
// captured sequence of substeps can be replayed as a graph.
#pragma once
#include "sim_kernels.hpp"

namespace tacchi {

struct BatchItem {
    int contact;
    int block;
};

// Per-contact constants of a batched substep (FP32 contacts).
struct BatchConsts {
    float dt, stress_coef, mscale, pscale, munit, punit;
};

// Each workgroup takes IPW consecutive work items (the tuner's items-per-
// workgroup setting), one after another, reusing its LDS; the barrier between
// two items lets the last LDS reads of one finish before the next overwrites.
// IPW is a template parameter: with a run-time count the loop around the
// inlined block code cost the one-item launches 50 % (measured).

// P2G of one substep; the first launch of the substep (bump != 0) advances the
// device substep counter, which the grid update then reads.
template <int B, int MODEL, int WG, int IPW>
__global__ void __launch_bounds__(WG) k_p2g_batch(const BatchItem *items, int nitems, const SimDev<float> *descs,
                                                  const BatchConsts *cc, int *step, int bump)
{
    if (bump && blockIdx.x == 0 && threadIdx.x == 0) *step += 1;
#pragma unroll
    for (int q = 0; q < IPW; ++q) {
        const int k = blockIdx.x * IPW + q;
        if (k >= nitems) return;
        if (q > 0) __syncthreads();
        const BatchItem it = items[k];
        const SimDev<float> S = descs[it.contact];
        const BatchConsts c = cc[it.contact];
        p2g_block<float, B, false, MODEL, WG>(S, it.block, 0.0f, c.mscale, c.pscale, c.munit, c.punit);
    }
}

template <int B, int WG, int IPW>
__global__ void __launch_bounds__(WG) k_grid_batch(const BatchItem *items, int nitems, const SimDev<float> *descs,
                                                   const BatchConsts *cc, const IndenterDev<double> *itab,
                                                   int nsteps, const int *step)
{
#pragma unroll
    for (int q = 0; q < IPW; ++q) {
        const int kk = blockIdx.x * IPW + q;
        if (kk >= nitems) return;
        if (q > 0) __syncthreads();
        const BatchItem it = items[kk];
        const SimDev<float> S = descs[it.contact];
        int k = *step;
        k = k < 0 ? 0 : (k >= nsteps ? nsteps - 1 : k);
        const IndenterDev<double> I = itab[(int64_t)it.contact * nsteps + k];
        grid_block<float, B, WG>(S, it.block, I, cc[it.contact].dt);
    }
}

// SORT: the substep's G2P first sorts each bin list by slot (as every
// kSortEvery-th single-contact G2P does).
template <int B, int MODEL, int WG, int IPW, bool SORT>
__global__ void __launch_bounds__(WG) k_g2p_batch(const BatchItem *items, int nitems, const SimDev<float> *descs,
                                                  const BatchConsts *cc)
{
#pragma unroll
    for (int q = 0; q < IPW; ++q) {
        const int k = blockIdx.x * IPW + q;
        if (k >= nitems) return;
        if (q > 0) __syncthreads();
        const BatchItem it = items[k];
        const SimDev<float> S = descs[it.contact];
        const BatchConsts c = cc[it.contact];
        g2p_block<float, B, MODEL, WG, SORT>(S, it.block, c.dt, c.stress_coef);
    }
}

}  // namespace tacchi
