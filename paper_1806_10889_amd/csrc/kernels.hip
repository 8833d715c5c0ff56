// kernels.hip -- the device kernels of one splitting step on gfx950, compiled
// ahead of time: the signalling operator S (its edge code in s_device.h),
// the step-counter advance, the regroup pass, and the launchers (the chi
// kernels with the generic network policy are compiled from
// chi_generic.hip).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "s_device.h"

namespace tissue_impl {

// ---------------------------------------------------------------------------
// S: one lane per edge
// ---------------------------------------------------------------------------
namespace {

// Workgroup b of n, dealt to XCD b mod 8, takes item x q + min(x, r) + b / 8
// (x = b mod 8, q = n / 8, r = n mod 8): each XCD gets one contiguous range
// of the items (a bijection on 0..n-1).
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t n)
{
    const uint32_t x = b % kXcds, k = b / kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + min(x, r) + k;
}

}  // namespace

// FIX = 2 or 1: every edge of the launch has face groups of FIX and FIX
// voxels (no LDS); FIX = 0: any sizes.
template <int FIX>
__global__ __launch_bounds__(kWave) void s_kernel(const DevTissue *const *tbl, const SItem *items,
                                                  uint32_t n_items, double dt, uint32_t kstep)
{
    __shared__ SShared sh;
    // one workgroup per item: consecutive items on one XCD (workgroups are
    // dealt to the XCDs in turn), so that the edges around a cell share that
    // XCD's L2
    const uint32_t it = xcd_contiguous(blockIdx.x, gridDim.x);
    if (it >= n_items) return;
    s_item<FIX>(tbl, items[it], dt, kstep, sh);
}

// step_base += n for every tissue of the table
__global__ void advance_kernel(DevTissue *const *tbl, uint32_t n_tissues, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_tissues) tbl[i]->step_base += n;
}

// ---------------------------------------------------------------------------
// Regroup: reorder the cells of one leaf-count class of one tissue by their
// total propensity after the last compact chi pass, largest first, in
// buckets of 1/16 of a binary order of magnitude below the class's largest,
// so that the cells of a work item (one wavefront) carry similar numbers of
// events and the heaviest items start first.  A cell's result depends only
// on its own counts and counters, never on its item or position.  One
// workgroup per segment (up to kRegroupChunk consecutive cells of a class
// of one tissue, whole work items): every thread holds its cells and their
// loads in registers, so the list is read once and rewritten in place.
// ---------------------------------------------------------------------------
constexpr int kRegroupThreads = 1024;
constexpr int kRegroupPerThread = (int)(kRegroupChunk / kRegroupThreads);
constexpr int kRegroupBuckets = 256;
static_assert(kRegroupChunk % kRegroupThreads == 0, "regroup chunk");

__global__ __launch_bounds__(kRegroupThreads) void regroup_kernel(const DevTissue *const *tbl,
                                                                  const ChiItem *segs,
                                                                  uint32_t n_segs)
{
    __shared__ uint32_t count[kRegroupBuckets];
    __shared__ uint32_t next[kRegroupBuckets];
    __shared__ uint32_t top_bits;
    if (blockIdx.x >= n_segs) return;
    const ChiItem seg = segs[blockIdx.x];
    const DevTissue *T = tbl[seg.tissue];
    int32_t *cl = T->cell_list + seg.first;
    const float *load = T->load;
    const uint32_t n = min(seg.count, kRegroupChunk);
    const int tid = threadIdx.x;
    for (int b = tid; b < kRegroupBuckets; b += kRegroupThreads) count[b] = 0u;
    if (tid == 0) top_bits = 0u;
    // this thread's cells and loads (non-negative floats order as their bits)
    int32_t cell[kRegroupPerThread];
    float key[kRegroupPerThread];
    uint32_t mb = 0u;
#pragma unroll
    for (int r = 0; r < kRegroupPerThread; ++r) {
        const uint32_t i = (uint32_t)(r * kRegroupThreads + tid);
        cell[r] = i < n ? cl[i] : 0;
        key[r] = i < n ? load[cell[r]] : 0.0f;
        mb = max(mb, __float_as_uint(key[r]));
    }
    __syncthreads();  // counters cleared; every cell read before any is rewritten
    atomicMax(&top_bits, mb);
    __syncthreads();
    const float top = __uint_as_float(top_bits);
    int bucket[kRegroupPerThread];  // 0 = heaviest
#pragma unroll
    for (int r = 0; r < kRegroupPerThread; ++r) {
        const float x = key[r];
        int b = kRegroupBuckets - 1;
        if (x > 0.0f && top > 0.0f) {
            const float d = 16.0f * __log2f(top / x);
            b = d < (float)(kRegroupBuckets - 1) ? (int)d : kRegroupBuckets - 1;
        }
        bucket[r] = b;
        if ((uint32_t)(r * kRegroupThreads + tid) < n) atomicAdd(&count[b], 1u);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0u;
        for (int b = 0; b < kRegroupBuckets; ++b) {
            next[b] = acc;
            acc += count[b];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRegroupPerThread; ++r)
        if ((uint32_t)(r * kRegroupThreads + tid) < n) cl[atomicAdd(&next[bucket[r]], 1u)] = cell[r];
}

hipError_t launch_regroup(hipStream_t stream, const DevTissue *const *tbl, const ChiItem *segs,
                          uint32_t n_segs)
{
    if (n_segs == 0) return hipSuccess;
    hipLaunchKernelGGL(regroup_kernel, dim3(n_segs), dim3(kRegroupThreads), 0, stream, tbl, segs,
                       n_segs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t chi_lds_bytes(int mode, int P, int S, int cells_per_item)
{
    if (mode == kChiRow) return 0;  // static LDS only
    // compact: cells of P > 16 leaves take P / 16 lanes each
    if (mode == kChiLane16) return lane16_lds_bytes(S, cells_per_item * compact_lanes(P));
    // per cell: the tree (2P doubles) and P*S counts, plus slack for the
    // species-slot reads past the last voxel
    return (size_t)cells_per_item * ((size_t)2 * P * 8 + ((size_t)P * S + kMaxSpecies) * 4);
}


// table sizes of a network: species slots 4 or 8, reactions rounded up to a
// multiple of 4, diffusion channels 0, 4 or 8
void chi_variant(int S, int R, int ND, int &SM, int &RM, int &NDM)
{
    SM = S <= 4 ? 4 : 8;
    RM = R <= 4 ? 4 : R <= 8 ? 8 : R <= 12 ? 12 : 16;
    NDM = ND == 0 ? 0 : ND <= 4 ? 4 : 8;
    if (NDM > SM) SM = NDM;
}

hipError_t launch_chi(int SM, int RM, int NDM, const ChiArgs &a)
{
    // each (species slots, diffusion slots) row of variants is compiled in
    // its own translation unit (chi_generic.hip built once per part)
    if (SM == 4 && NDM == 0) return launch_chi_part0(RM, a);
    if (SM == 4 && NDM == 4) return launch_chi_part1(RM, a);
    if (SM == 8 && NDM == 0) return launch_chi_part2(RM, a);
    if (SM == 8 && NDM == 4) return launch_chi_part3(RM, a);
    if (SM == 8 && NDM == 8) return launch_chi_part4(RM, a);
    return hipErrorInvalidValue;
}

hipError_t launch_s(hipStream_t stream, const DevTissue *const *tbl, const SItem *items,
                    uint32_t n_items, double dt, uint32_t kstep, int fix)
{
    if (fix == 2)
        hipLaunchKernelGGL(s_kernel<2>, dim3(n_items), dim3(kWave), 0, stream, tbl, items, n_items,
                           dt, kstep);
    else if (fix == 1)
        hipLaunchKernelGGL(s_kernel<1>, dim3(n_items), dim3(kWave), 0, stream, tbl, items, n_items,
                           dt, kstep);
    else
        hipLaunchKernelGGL(s_kernel<0>, dim3(n_items), dim3(kWave), 0, stream, tbl, items, n_items,
                           dt, kstep);
    return hipGetLastError();
}

hipError_t launch_advance(hipStream_t stream, DevTissue *const *tbl, uint32_t n_tissues,
                          uint32_t n)
{
    const uint32_t threads = 256;
    hipLaunchKernelGGL(advance_kernel, dim3((n_tissues + threads - 1) / threads), dim3(threads), 0,
                       stream, tbl, n_tissues, n);
    return hipGetLastError();
}

}  // namespace tissue_impl
