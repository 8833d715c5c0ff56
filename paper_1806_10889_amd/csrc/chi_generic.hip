// chi_generic.hip -- the chi kernels with the generic (runtime-table) network
// policy, compiled ahead of time for gfx950.  The build compiles this file
// once per part (TISSUE_GENERIC_PART = 0..4), each part holding one row of
// table sizes (species slots, diffusion slots) for every reaction-slot
// count, so that the parts compile in parallel; launch_chi (kernels.hip)
// dispatches to the part of a network's table sizes.
#include <hip/hip_runtime.h>

#include "chi_kernels.h"
#include "kernels.h"

#ifndef TISSUE_GENERIC_PART
#error "TISSUE_GENERIC_PART must be defined (0..4)"
#endif

namespace tissue_impl {

// chi with the generic (runtime-table) network policy
template <int SM, int RM, int NDM>
__global__ __launch_bounds__(kWave) void chi_lane_kernel(const DevTissue *const *tbl,
                                                         const ChiItem *items, uint32_t n_items,
                                                         uint32_t *queue, int persistent,
                                                         int cells_per_item, int log2p, double dt,
                                                         uint32_t kstep, uint32_t tag,
                                                         uint32_t *n_items_dev, int prio)
{
    extern __shared__ __align__(16) unsigned char lds[];
    chi_lane_body<NetGeneric<SM, RM, NDM>>(lds, tbl, items, n_items, queue, persistent,
                                           cells_per_item, log2p, dt, kstep, tag, n_items_dev, prio,
                                           blockIdx.x);
}

template <int SM, int RM, int NDM, int G>
__global__ __launch_bounds__(kWave) void chi_lane16_kernel(const DevTissue *const *tbl,
                                                           const ChiItem *items, uint32_t n_items,
                                                           uint32_t *queue, int persistent,
                                                           int cells_per_item, double dt,
                                                           uint32_t kstep, uint32_t tag,
                                                           ChiItem *retry_items, uint32_t *retry_count,
                                                           int prio)
{
    extern __shared__ __align__(16) unsigned char lds[];
    chi_lane16_body<NetGeneric<SM, RM, NDM>, G>(lds, tbl, items, n_items, queue, persistent,
                                                cells_per_item, dt, kstep, tag, retry_items,
                                                retry_count, prio);
}

template <int SM, int RM, int NDM, int RW>
__global__ __launch_bounds__(kWave) void chi_row_kernel(const DevTissue *const *tbl,
                                                        const ChiItem *items, uint32_t n_items,
                                                        uint32_t *queue, int persistent, double dt,
                                                        uint32_t kstep, uint32_t tag, int prio)
{
    __shared__ RowShared sh;
    chi_row_body<NetGeneric<SM, RM, NDM>, RW>(sh, tbl, items, n_items, queue, persistent, dt,
                                              kstep, tag, prio);
}

namespace {

int log2_exact(int P)
{
    int l = 0;
    while ((1 << l) < P) ++l;
    return l;
}

template <int SM, int RM, int NDM>
hipError_t launch_variant(const ChiArgs &a)
{
    if (a.mode == kChiRow && a.rw == 64) {
        hipLaunchKernelGGL((chi_row_kernel<SM, RM, NDM, 64>), dim3(a.grid), dim3(kWave), 0, a.stream,
                           a.tbl, a.items, a.n_items, a.queue, a.persistent, a.dt, a.kstep, a.tag, a.prio);
    } else if (a.mode == kChiRow && a.rw == 32) {
        hipLaunchKernelGGL((chi_row_kernel<SM, RM, NDM, 32>), dim3(a.grid), dim3(kWave), 0, a.stream,
                           a.tbl, a.items, a.n_items, a.queue, a.persistent, a.dt, a.kstep, a.tag, a.prio);
    } else if (a.mode == kChiRow) {
        hipLaunchKernelGGL((chi_row_kernel<SM, RM, NDM, 16>), dim3(a.grid), dim3(kWave), 0, a.stream,
                           a.tbl, a.items, a.n_items, a.queue, a.persistent, a.dt, a.kstep, a.tag, a.prio);
    } else if (a.mode == kChiLane16 && a.P == 64) {
        hipLaunchKernelGGL((chi_lane16_kernel<SM, RM, NDM, 4>), dim3(a.grid), dim3(kWave), a.lds,
                           a.stream, a.tbl, a.items, a.n_items, a.queue, a.persistent,
                           a.cells_per_item, a.dt, a.kstep, a.tag, a.retry_items, a.retry_count, a.prio);
    } else if (a.mode == kChiLane16 && a.P == 32) {
        hipLaunchKernelGGL((chi_lane16_kernel<SM, RM, NDM, 2>), dim3(a.grid), dim3(kWave), a.lds,
                           a.stream, a.tbl, a.items, a.n_items, a.queue, a.persistent,
                           a.cells_per_item, a.dt, a.kstep, a.tag, a.retry_items, a.retry_count, a.prio);
    } else if (a.mode == kChiLane16 && a.P <= 16) {
        hipLaunchKernelGGL((chi_lane16_kernel<SM, RM, NDM, 1>), dim3(a.grid), dim3(kWave), a.lds,
                           a.stream, a.tbl, a.items, a.n_items, a.queue, a.persistent,
                           a.cells_per_item, a.dt, a.kstep, a.tag, a.retry_items, a.retry_count, a.prio);
    } else if (a.mode == kChiLane16) {
        return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((chi_lane_kernel<SM, RM, NDM>), dim3(a.grid), dim3(kWave), a.lds,
                           a.stream, a.tbl, a.items, a.n_items, a.queue, a.persistent,
                           a.cells_per_item, log2_exact(a.P), a.dt, a.kstep, a.tag, a.n_items_dev, a.prio);
    }
    return hipGetLastError();
}

}  // namespace

#if TISSUE_GENERIC_PART == 0
constexpr int kPartSM = 4, kPartNDM = 0;
#define TISSUE_PART_FN launch_chi_part0
#elif TISSUE_GENERIC_PART == 1
constexpr int kPartSM = 4, kPartNDM = 4;
#define TISSUE_PART_FN launch_chi_part1
#elif TISSUE_GENERIC_PART == 2
constexpr int kPartSM = 8, kPartNDM = 0;
#define TISSUE_PART_FN launch_chi_part2
#elif TISSUE_GENERIC_PART == 3
constexpr int kPartSM = 8, kPartNDM = 4;
#define TISSUE_PART_FN launch_chi_part3
#elif TISSUE_GENERIC_PART == 4
constexpr int kPartSM = 8, kPartNDM = 8;
#define TISSUE_PART_FN launch_chi_part4
#else
#error "TISSUE_GENERIC_PART out of range"
#endif

hipError_t TISSUE_PART_FN(int RM, const ChiArgs &a)
{
    if (RM == 4) return launch_variant<kPartSM, 4, kPartNDM>(a);
    if (RM == 8) return launch_variant<kPartSM, 8, kPartNDM>(a);
    if (RM == 12) return launch_variant<kPartSM, 12, kPartNDM>(a);
    if (RM == 16) return launch_variant<kPartSM, 16, kPartNDM>(a);
    return hipErrorInvalidValue;
}

}  // namespace tissue_impl
